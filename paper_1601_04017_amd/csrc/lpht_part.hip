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
// bits and then 16 sub-buckets of the next 4 bits inside each, so that a
// workgroup's scatter has few open output runs at a time and its writes
// complete whole lines in L2 (one level of 4096 buckets left each XCD's L2
// with far more partly written lines than it holds).  Skewed streams put one
// key on most lanes of a wavefront, so the LDS atomics of all passes first
// combine the lanes that share the leading lane's bucket or key.  Each level is a count
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
constexpr uint32_t kMaxBits = 12;       // at most 4096 buckets in all
constexpr uint32_t kCountWG = 512;      // workgroups of the count and scatter passes
constexpr uint32_t kCountThreads = 512;
constexpr uint32_t kApplyThreads = 1024;
constexpr uint32_t kItemOps = 32768;    // operations per apply work item
// LDS combining slots: 8192 of 16 B (128 KiB, one workgroup per CU) hold the
// ~4.4k distinct keys of a bucket of a 10^8-key Zipf(1) batch; with flags
// each slot also keeps its representative's index, and 4096 slots fit
constexpr uint32_t kSlotsNoFlags = 8192;
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
  // kUnroll independent loads per lane before any is used: enough bytes in
  // flight to cover the memory latency
  for (u64 base = lo; base < hi; base += (u64)blockDim.x * kUnroll) {
    u64 key[kUnroll];
#pragma unroll
    for (uint32_t j = 0; j < kUnroll; ++j) {
      const u64 i = base + (u64)j * blockDim.x + threadIdx.x;
      key[j] = i < hi ? part_key<L>(V.skeys, i) : 0;
    }
#pragma unroll
    for (uint32_t j = 0; j < kUnroll; ++j) {
      const u64 i = base + (u64)j * blockDim.x + threadIdx.x;
      bool act = i < hi;
      if (act && lv == 0) {
        if (key[j] == kEmpty || key[j] == kTomb) {
          err |= kErrReserved;
          if (A.flags) A.flags[i] = 0xFE;
          act = false;
        } else if (A.flags) {
          A.flags[i] = 0;
        }
      }
      const uint32_t b = act ? (uint32_t)(hash_of<L>(T, key[j], A.crc_hi, A.crc_lo, A.mul) >> (64 - V.bits)) : 0;
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
// and (with V.items) the first work item of each bucket.
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
      if (V.items) V.items[b] = (uint32_t)it;
      e += tot[j];
      it += (tot[j] + kItemOps - 1) / kItemOps;
    }
  }
  if (threadIdx.x == 0) {
    V.btot[V.nb] = etotal;
    if (V.items) V.items[V.nb] = (uint32_t)itotal;
  }
}

template <int L>
__global__ void __launch_bounds__(kCountThreads) k_part_scatter(PartK k, uint32_t lv) {
  __shared__ uint32_t T[8][256];
  __shared__ u64 cur[1u << kMaxBits];
  crc_tables_build(T);
  const Level &V = k.L[lv];
  const BulkArgs &A = k.A;
  const u64 n = lv == 0 ? A.n : k.L[0].btot[k.L[0].nb];
  const u64 lo = (u64)blockIdx.x * k.chunk;
  const u64 hi = lo + k.chunk < n ? lo + k.chunk : n;
  // only the buckets this share touched hold a valid reservation; the others
  // are never used below
  for (uint32_t b = threadIdx.x; b < V.nb; b += blockDim.x) cur[b] = V.btot[b] + V.hist[(u64)blockIdx.x * V.nb + b];
  __syncthreads();
  for (u64 base = lo; base < hi; base += (u64)blockDim.x * kUnroll) {
    u64 key[kUnroll], val[kUnroll];
    uint32_t idx[kUnroll];
#pragma unroll
    for (uint32_t j = 0; j < kUnroll; ++j) {
      const u64 i = base + (u64)j * blockDim.x + threadIdx.x;
      const bool in = i < hi;
      key[j] = in ? part_key<L>(V.skeys, i) : 0;
      val[j] = in && V.dvals ? part_key<L>(V.svals, i) : 0;
      idx[j] = in && V.didx ? (V.sidx ? V.sidx[i] : (uint32_t)i) : 0;
    }
#pragma unroll
    for (uint32_t j = 0; j < kUnroll; ++j) {
      const u64 i = base + (u64)j * blockDim.x + threadIdx.x;
      const bool valid = i < hi && !(lv == 0 && (key[j] == kEmpty || key[j] == kTomb));
      const uint32_t b = valid ? (uint32_t)(hash_of<L>(T, key[j], A.crc_hi, A.crc_lo, A.mul) >> (64 - V.bits)) : 0;
      bool act = valid;
      u64 pos = 0;
      for (int r = 0; r < kAggRounds; ++r) {
        u64 lt = 0;
        uint32_t ll = 0;
        const u64 m = match_first(act, b, lt, ll);
        if (__popcll(m) < 2) break;
        u64 at = 0;
        if ((threadIdx.x & 63) == ll) at = atomicAdd((unsigned long long *)&cur[(uint32_t)lt], (u64)__popcll(m));
        at = __shfl(at, (int)ll, 64);
        if ((m >> (threadIdx.x & 63)) & 1) {
          pos = at + lanes_below(m);
          act = false;
        }
      }
      if (act) pos = atomicAdd((unsigned long long *)&cur[b], 1ull);
      if (!valid) continue;
      part_store<L>(V.dkeys, pos, key[j]);
      if (V.dvals) part_store<L>(V.dvals, pos, val[j]);
      if (V.didx) V.didx[pos] = idx[j];
    }
  }
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
__global__ void __launch_bounds__(kApplyThreads) k_part_apply(PartK k) {
  constexpr uint32_t S = FL ? kSlotsFlags : kSlotsNoFlags;
  constexpr uint32_t SB = FL ? 12 : 13;
  static_assert((1u << SB) == S, "slot bits");
  __shared__ uint32_t T[8][256];
  __shared__ u64 s_key[S];
  __shared__ u64 s_sum[S];
  __shared__ uint32_t s_rep[FL ? S : 1];
  __shared__ uint32_t s_claims;
  __shared__ uint32_t s_item[2];
  __shared__ long long s_acc[2];
  __shared__ uint32_t s_err;
  crc_tables_build(T);
  for (uint32_t q = threadIdx.x; q < S; q += blockDim.x) {
    s_key[q] = 0;
    s_sum[q] = 0;
    if (FL) s_rep[q] = ~0u;
  }
  const BulkArgs &A = k.A;
  const Level &V = k.L[1];
  long long d_used = 0, d_live = 0;
  uint32_t err = 0;
  const uint32_t nitems = V.items[V.nb];
  for (uint32_t j = blockIdx.x; j < nitems; j += gridDim.x) {
    if (threadIdx.x == 0) {
      // the bucket of item j: the last b with items[b] <= j
      uint32_t a = 0, z = V.nb;  // items[a] <= j < items[z]
      while (z - a > 1) {
        const uint32_t m = (a + z) / 2;
        if (V.items[m] <= j)
          a = m;
        else
          z = m;
      }
      s_item[0] = a;
      s_item[1] = V.items[a + 1] - V.items[a] == 1;
      s_claims = 0;
    }
    __syncthreads();
    const uint32_t b = s_item[0];
    const bool alone = s_item[1] != 0;
    const u64 lo = V.btot[b] + (u64)(j - V.items[b]) * kItemOps;
    const u64 end = V.btot[b + 1];
    const u64 hi = lo + kItemOps < end ? lo + kItemOps : end;
    for (u64 pb = lo; pb < hi; pb += (u64)blockDim.x * kUnroll) {
     u64 keys[kUnroll], ds[kUnroll];
     uint32_t idxs[kUnroll];
#pragma unroll
     for (uint32_t j = 0; j < kUnroll; ++j) {
       const u64 p = pb + (u64)j * blockDim.x + threadIdx.x;
       const bool in = p < hi;
       keys[j] = in ? part_key<L>(V.dkeys, p) : 0;
       ds[j] = in ? (V.dvals ? part_key<L>(V.dvals, p) : 1) : 0;
       idxs[j] = in && FL ? V.didx[p] : 0;
     }
     for (uint32_t j = 0; j < kUnroll; ++j) {
      // equal keys on the lanes of this step first (a batch key is never 0
      // here, so 0 marks lanes past the end)
      bool act = keys[j] != 0;
      bool open = act;  // not yet in a group
      const u64 key = keys[j];
      u64 d = ds[j];
      uint32_t idx = idxs[j];
      // every lane runs every round (the shuffles read all lanes)
      for (int r = 0; r < kAggRounds; ++r) {
        u64 lk = 0;
        uint32_t ll = 0;
        const u64 m = match_first(open, key, lk, ll);
        if (__popcll(m) < 2) break;
        const bool in = (m >> (threadIdx.x & 63)) & 1;
        const u64 sum = (u64)wave_sum(in ? (long long)d : 0);
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
  }
  flush_counts(A.status, d_used, d_live, err, s_acc, &s_err);
}

struct Carved {
  size_t btot[2], hist[2], items, keys[2], vals[2], idx[2], total;
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
  const uint32_t apply_grid = std::max<uint32_t>(1, num_cus);  // one workgroup per CU (LDS)
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
    LPHT_PART(k_part_scatter, k.nwg, kCountThreads, k, lv);
#undef LPHT_PART
  }
  if (a.flags) {
    if (a.layout == 0)
      hipLaunchKernelGGL((k_part_apply<0, true>), dim3(apply_grid), dim3(kApplyThreads), 0, s, k);
    else
      hipLaunchKernelGGL((k_part_apply<1, true>), dim3(apply_grid), dim3(kApplyThreads), 0, s, k);
  } else {
    if (a.layout == 0)
      hipLaunchKernelGGL((k_part_apply<0, false>), dim3(apply_grid), dim3(kApplyThreads), 0, s, k);
    else
      hipLaunchKernelGGL((k_part_apply<1, false>), dim3(apply_grid), dim3(kApplyThreads), 0, s, k);
  }
  return hipGetLastError();
}

}  // namespace lpht
