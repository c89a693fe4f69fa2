// Sort-based bulk build and batched merge of liblpht (Sec. 5.5).
//
// The batch (and, for a merge, the table's live elements, which count as
// earlier than every batch entry) is ordered by hash value; among equal keys
// all but the last are removed (with "add", the kept one carries the sum of
// all their values); the result is laid into an empty table as if inserted
// one by one in that order, so every element starts its search for a free
// cell at the larger of its home and the previous element's position.  The
// table that results is a function of the key set alone.
//
// Order: by u = the upper 32 hash bits (the lower half is a function of u, as
// both halves are the same CRC with different seed constants), then by key,
// then by sequence number (0 for the table's elements, i + 1 for batch entry
// i).  The home position is the top log2 c bits of u.
//
// The target table is cut into blocks of B = 256 cells.  Steps:
//   A. partition by the top l1 bits of the block index (<= 1024 bins): each
//      workgroup counts its contiguous share of the input per bin
//      (k_bm_count), scans give every (bin, workgroup) pair its own output
//      range (k_bm_scan_rows, k_bm_scan_bins), and each workgroup writes its
//      share in tiles of 1024 elements, equal keys of a tile combined in an
//      LDS hash table (k_bm_scatter), the entries freed by combining marked
//      with the empty key -- no global atomics;
//   B. one workgroup per first-level bin partitions its elements by the
//      remaining l2 bits into blocks (k_bm_partition), combining equal keys
//      again per chunk of 1024 elements, so a hot key reaches its block at
//      most once per chunk;
//   C. one wavefront per block sorts the block's elements in LDS (bitonic,
//      k_bm_block_wave; a workgroup for blocks of more than 256 elements,
//      k_bm_block), removes equal keys and computes the block's carry
//      function: the number of elements that run past the block's end is
//      f(c) = max(a, c + m - B) when c elements run in from the left, with m
//      the block's distinct keys and a = max(0, m + max_k(pos_k - k) - s - B)
//      (s = the block's first cell, pos_k the home of its k-th element);
//      blocks with more elements than LDS holds go to k_bm_big_block, which
//      sorts in global memory;
//   D. the carry functions compose as max-plus maps; a scan over the blocks
//      (k_bm_scan_reduce, k_bm_scan_top, k_bm_scan_down) gives every block
//      its carry-in and the carry out of the last block (the elements that
//      wrap);
//   E. each block places its elements at p_k = k + max(s + c_in,
//      max_{l<=k}(pos_l - l)) (k_bm_place): cells of its own block go through
//      an LDS image written once, empty cells included, except the first
//      c_in cells, which belong to elements of earlier blocks that write them
//      themselves;
//   F. the wrapped elements, the largest in the order, take the first free
//      cells from cell 0 on (k_bm_wrap).

#include <hip/hip_runtime.h>

#include <mutex>

#include <algorithm>
#include <climits>
#include <type_traits>

#include "lpht_bulk.h"
#include "lpht_device.h"

namespace lpht {

namespace {

constexpr uint32_t kTileA = 1024;   // stage A tile (elements)
constexpr uint32_t kSlots = 2048;   // LDS combining table slots (>= 2 x elements combined)
constexpr uint32_t kL1Max = 1024;
constexpr uint32_t kL2Max = 2048;
constexpr uint32_t kGAMax = 1024;
constexpr uint32_t kEW = 256;       // elements a wavefront sorts in LDS in stage C
constexpr uint32_t kEMax = 1024;    // elements a workgroup sorts in LDS in stage C
constexpr uint32_t kScanPer = 16;   // blocks per thread in stage D
constexpr uint32_t kScanTile = 256 * kScanPer;

template <int L>
using KT = typename std::conditional<L == 0, uint32_t, u64>::type;

struct BmK {
  uint32_t layout, op;
  const void *old_cells;
  uint64_t cold;  // old cells scanned (element indices below are old cells)
  const void *keys, *vals;
  uint64_t n, ntot;
  void *cells;
  uint32_t log2c, log2b, nb_bits, l1_bits, l2_bits, L1, GA;
  uint64_t c, nblocks, per, ntiles;
  uint64_t cap_items;  // staging entries (an upper bound of the elements)
  uint32_t crc_hi, crc_lo;
  u64 mul;             // nonzero: multiplicative hash
  DevStatus *st;
  BulkMergeCtl *ctl;
  void *keyA, *valA;
  uint32_t *seqA;
  void *keyB, *valB;
  uint32_t *seqB;
  uint32_t *mcnt, *moff, *l1_off, *blk_off, *blk_cnt, *big_list, *mid_list;
  long long *car_a, *car_d, *cin, *tile_a, *tile_d;
};

__device__ __forceinline__ uint32_t top_bits(uint32_t u, uint32_t bits) { return bits ? u >> (32 - bits) : 0u; }

// The upper 32 bits of the table's hash: the sort key (ties broken by key),
// holding every position bit of a table of up to 2^32 cells.
template <int L>
__device__ __forceinline__ uint32_t sort_hash(const uint32_t (*T)[256], KT<L> k, uint32_t crc_hi, u64 mul) {
  if (mul) return (uint32_t)(((u64)k * mul) >> 32);
  const uint32_t c = (L == 0) ? crc0_u32(T, (uint32_t)k) : crc0_u64(T, (u64)k);
  return c ^ crc_hi;
}

// Element e of the input: old cell e (e < cold; live cells only) or batch
// entry e - cold (reserved keys are skipped and reported).
template <int L>
__device__ __forceinline__ bool load_elem(const BmK &k, u64 e, KT<L> &key, KT<L> &val, uint32_t &seq,
                                          uint32_t &err) {
  if (e < k.cold) {
    if (L == 0) {
      const u64 w = ((const u64 *)k.old_cells)[e];
      key = (KT<L>)(w & 0xFFFFFFFFull);
      val = (KT<L>)(w >> 32);
    } else {
      const u64x2 w = ((const u64x2 *)k.old_cells)[e];
      key = (KT<L>)w.x;
      val = (KT<L>)w.y;
    }
    seq = 0;
    return (u64)key > kTomb;
  }
  const u64 i = e - k.cold;
  key = ((const KT<L> *)k.keys)[i];
  val = k.vals ? ((const KT<L> *)k.vals)[i] : (KT<L>)1;
  seq = (uint32_t)(i + 1);
  if ((u64)key <= kTomb) {
    err |= kErrReserved;
    return false;
  }
  return true;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane >= (uint32_t)o) v += t;
  }
  return v;
}

// Exclusive scan over the workgroup (<= 16 wavefronts); sw holds >= 17 words.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total, uint32_t *sw) {
  const uint32_t incl = wave_incl_scan(v);
  const uint32_t w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 63) sw[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (uint32_t i = 0; i < nw; ++i) {
      const uint32_t t = sw[i];
      sw[i] = acc;
      acc += t;
    }
    sw[nw] = acc;
  }
  __syncthreads();
  const uint32_t r = sw[w] + incl - v;
  *total = sw[nw];
  __syncthreads();
  return r;
}

// Inclusive max-scan over the workgroup; sm holds >= 17 entries.
__device__ __forceinline__ long long block_incl_max(long long v, long long *total, long long *sm) {
  const uint32_t lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long t = __shfl_up(v, o, 64);
    if (lane >= (uint32_t)o) v = v > t ? v : t;
  }
  const uint32_t w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 63) sm[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long acc = LLONG_MIN;
    for (uint32_t i = 0; i < nw; ++i) {
      const long long t = sm[i];
      sm[i] = acc;
      acc = acc > t ? acc : t;
    }
    sm[nw] = acc;
  }
  __syncthreads();
  const long long r = v > sm[w] ? v : sm[w];
  *total = sm[nw];
  __syncthreads();
  return r;
}

// Max-plus carry maps f(c) = max(a, c + d); then(x, y) = apply x, then y.
struct Carry {
  long long a, d;
};
__device__ __forceinline__ Carry then(Carry x, Carry y) {
  Carry r;
  const long long t = x.a + y.d;
  r.a = y.a > t ? y.a : t;
  r.d = x.d + y.d;
  return r;
}

// LDS combining of equal keys: slot table with linear probing on u.
template <int L>
struct Combine {
  KT<L> key[kSlots];
  KT<L> val[kSlots];
  uint32_t seq[kSlots];
};

template <int L>
__device__ __forceinline__ void combine_clear(Combine<L> &cb) {
  for (uint32_t i = threadIdx.x; i < kSlots; i += blockDim.x) {
    cb.key[i] = 0;
    cb.val[i] = 0;
    cb.seq[i] = 0;
  }
}

template <int L>
__device__ __forceinline__ uint32_t combine_claim(Combine<L> &cb, KT<L> key, uint32_t u) {
  uint32_t p = u & (kSlots - 1);
  for (;;) {
    const KT<L> prev = atomicCAS(&cb.key[p], (KT<L>)0, key);
    if (prev == 0 || prev == key) return p;
    p = (p + 1) & (kSlots - 1);
  }
}

// After every element has claimed its slot (and a barrier): assign keeps the
// value of the largest sequence number, add sums.
template <int L>
__device__ __forceinline__ void combine_values(Combine<L> &cb, bool ok, uint32_t p, KT<L> val, uint32_t seq,
                                               uint32_t op) {
  if (ok) {
    atomicMax(&cb.seq[p], seq);
    if (op == 1) atomicAdd(&cb.val[p], val);
  }
  __syncthreads();
  if (ok && op == 0 && cb.seq[p] == seq) cb.val[p] = val;
}

// ------------------------------------------------------------- stage A

__global__ void k_bm_init(BulkMergeCtl *ctl) {
  if (threadIdx.x < sizeof(BulkMergeCtl) / 8) ((unsigned long long *)ctl)[threadIdx.x] = 0;
}

template <int L>
__global__ void __launch_bounds__(256) k_bm_count(BmK k) {
  __shared__ uint32_t T[8][256];
  __shared__ uint32_t hist[kL1Max];
  __shared__ uint32_t s_err;
  crc_tables_build(T);
  for (uint32_t i = threadIdx.x; i < k.L1; i += blockDim.x) hist[i] = 0;
  if (threadIdx.x == 0) s_err = 0;
  __syncthreads();
  const u64 lo = (u64)blockIdx.x * k.per;
  const u64 hi = std::min<u64>(lo + k.per, k.ntot);
  uint32_t err = 0;
  for (u64 e = lo + threadIdx.x; e < hi; e += blockDim.x) {
    KT<L> key, val;
    uint32_t seq;
    if (!load_elem<L>(k, e, key, val, seq, err)) continue;
    atomicAdd(&hist[top_bits(sort_hash<L>(T, key, k.crc_hi, k.mul), k.l1_bits)], 1u);
  }
  if (err) atomicOr(&s_err, err);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < k.L1; i += blockDim.x) k.mcnt[(u64)i * k.GA + blockIdx.x] = hist[i];
  if (threadIdx.x == 0 && s_err) atomicOr(&k.st->err, s_err);
}

// One workgroup per bin: exclusive scan of the bin's per-workgroup counts
// (offsets inside the bin) and the bin's total.
__global__ void __launch_bounds__(256) k_bm_scan_rows(BmK k) {
  __shared__ uint32_t sw[17];
  const uint32_t b = blockIdx.x;
  const uint32_t per = (k.GA + blockDim.x - 1) / blockDim.x;
  const uint32_t w0 = std::min(k.GA, threadIdx.x * per), w1 = std::min(k.GA, w0 + per);
  const u64 row = (u64)b * k.GA;
  uint32_t sum = 0;
  for (uint32_t w = w0; w < w1; ++w) sum += k.mcnt[row + w];
  uint32_t total;
  uint32_t acc = block_excl_scan(sum, &total, sw);
  for (uint32_t w = w0; w < w1; ++w) {
    k.moff[row + w] = acc;
    acc += k.mcnt[row + w];
  }
  if (threadIdx.x == 0) k.l1_off[b] = total;  // the bin's size; turned into its offset next
}

// One workgroup of 1024 threads: exclusive scan of the bin sizes.
__global__ void __launch_bounds__(1024) k_bm_scan_bins(BmK k) {
  __shared__ uint32_t sw[17];
  const uint32_t per = (k.L1 + blockDim.x - 1) / blockDim.x;
  const uint32_t b0 = std::min(k.L1, threadIdx.x * per), b1 = std::min(k.L1, b0 + per);
  uint32_t sum = 0;
  for (uint32_t b = b0; b < b1; ++b) sum += k.l1_off[b];
  uint32_t total;
  uint32_t acc = block_excl_scan(sum, &total, sw);
  for (uint32_t b = b0; b < b1; ++b) {
    const uint32_t t = k.l1_off[b];
    k.l1_off[b] = acc;
    acc += t;
  }
  if (threadIdx.x == 0) {
    k.l1_off[k.L1] = total;
    // more elements than the staging holds would mean inconsistent counts:
    // stop every later stage
    if (total > k.cap_items) k.ctl->full = 2;
  }
}

template <int L>
__global__ void __launch_bounds__(256) k_bm_scatter(BmK k) {
  __shared__ uint32_t T[8][256];
  __shared__ Combine<L> cb;
  __shared__ uint32_t cur[kL1Max];
  __shared__ uint32_t toff[kL1Max + 1];
  __shared__ uint16_t order[kTileA];
  __shared__ uint16_t obin[kTileA];
  __shared__ uint32_t sw[17];
  if (k.ctl->full) return;
  crc_tables_build(T);
  const uint32_t w = blockIdx.x;
  for (uint32_t i = threadIdx.x; i < k.L1; i += blockDim.x) cur[i] = k.l1_off[i] + k.moff[(u64)i * k.GA + w];
  const u64 lo = (u64)w * k.per;
  const u64 hi = std::min<u64>(lo + k.per, k.ntot);
  KT<L> *keyA = (KT<L> *)k.keyA;
  KT<L> *valA = (KT<L> *)k.valA;
  uint32_t err = 0;
  for (u64 tile = lo; tile < hi; tile += kTileA) {
    combine_clear<L>(cb);
    for (uint32_t i = threadIdx.x; i <= k.L1; i += blockDim.x) toff[i] = 0;
    __syncthreads();
    bool ok[4];
    uint32_t slot[4], sq[4];
    KT<L> vv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const u64 e = tile + threadIdx.x + 256 * j;
      KT<L> key = 0;
      ok[j] = e < hi && load_elem<L>(k, e, key, vv[j], sq[j], err);
      slot[j] = ok[j] ? combine_claim<L>(cb, key, sort_hash<L>(T, key, k.crc_hi, k.mul)) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (ok[j]) {
        atomicMax(&cb.seq[slot[j]], sq[j]);
        if (k.op == 1) atomicAdd(&cb.val[slot[j]], vv[j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (ok[j] && k.op == 0 && cb.seq[slot[j]] == sq[j]) cb.val[slot[j]] = vv[j];
    // bins of the combined elements, and their rank inside the tile's bin
    uint32_t bin[8], rk[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t i = threadIdx.x + 256 * j;
      bin[j] = ~0u;
      if (cb.key[i] != 0) {
        bin[j] = top_bits(sort_hash<L>(T, cb.key[i], k.crc_hi, k.mul), k.l1_bits);
        rk[j] = atomicAdd(&toff[bin[j]], 1u);
      }
    }
    __syncthreads();
    // exclusive scan of the per-bin counts of this tile (toff[L1] = total)
    {
      const uint32_t per = (k.L1 + 1 + blockDim.x - 1) / blockDim.x;
      const uint32_t b0 = std::min(k.L1 + 1, threadIdx.x * per), b1 = std::min(k.L1 + 1, b0 + per);
      uint32_t s = 0;
      for (uint32_t b = b0; b < b1; ++b) s += toff[b];
      uint32_t tot;
      uint32_t acc = block_excl_scan(s, &tot, sw);
      for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t t = toff[b];
        toff[b] = acc;
        acc += t;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (bin[j] != ~0u) {
        const uint32_t at = toff[bin[j]] + rk[j];
        order[at] = (uint16_t)(threadIdx.x + 256 * j);
        obin[at] = (uint16_t)bin[j];
      }
    }
    __syncthreads();
    // consecutive threads write consecutive positions of one bin's range
    const uint32_t total = toff[k.L1];
    for (uint32_t at = threadIdx.x; at < total; at += blockDim.x) {
      const uint32_t sl = order[at], b = obin[at];
      const u64 p = (u64)cur[b] + (at - toff[b]);
      keyA[p] = cb.key[sl];
      valA[p] = cb.val[sl];
      k.seqA[p] = cb.seq[sl];
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < k.L1; b += blockDim.x) cur[b] += toff[b + 1] - toff[b];
    __syncthreads();
  }
  // the entries of each (bin, workgroup) range left free by combined
  // duplicates get the empty key, which stage B skips
  for (uint32_t i = threadIdx.x; i < k.L1; i += blockDim.x) {
    const u64 m = (u64)i * k.GA + w;
    const u64 end = (u64)k.l1_off[i] + k.moff[m] + k.mcnt[m];
    for (u64 p = cur[i]; p < end; ++p) keyA[p] = 0;
  }
  if (err) atomicOr(&k.st->err, err);
}

// ------------------------------------------------------------- stage B

// One workgroup of 1024 threads per first-level bin s.
template <int L>
__global__ void __launch_bounds__(1024) k_bm_partition(BmK k) {
  __shared__ uint32_t T[8][256];
  __shared__ uint32_t hist[kL2Max];
  __shared__ Combine<L> cb;
  __shared__ uint32_t sw[17];
  if (k.ctl->full) return;
  crc_tables_build(T);
  const uint32_t s = blockIdx.x;
  const uint32_t nl2 = 1u << k.l2_bits;
  const uint32_t mask2 = nl2 - 1;
  for (uint32_t i = threadIdx.x; i < nl2; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  // the bin's stage-A range; entries with the empty key are holes
  const u64 out0 = k.l1_off[s];
  const uint32_t total = k.l1_off[s + 1] - k.l1_off[s];
  const KT<L> *keyA = (const KT<L> *)k.keyA;
  const KT<L> *valA = (const KT<L> *)k.valA;
  KT<L> *keyB = (KT<L> *)k.keyB;
  KT<L> *valB = (KT<L> *)k.valB;
  for (uint32_t j = threadIdx.x; j < total; j += blockDim.x) {
    const KT<L> key = keyA[out0 + j];
    if (key == 0) continue;
    atomicAdd(&hist[top_bits(sort_hash<L>(T, key, k.crc_hi, k.mul), k.nb_bits) & mask2], 1u);
  }
  __syncthreads();
  // block regions inside the bin's output range, sized by the raw counts
  uint32_t my_off[2] = {0, 0};
  {
    const uint32_t per = (nl2 + blockDim.x - 1) / blockDim.x;  // <= 2
    const uint32_t i0 = std::min(nl2, threadIdx.x * per), i1 = std::min(nl2, i0 + per);
    uint32_t sum = 0;
    for (uint32_t i = i0; i < i1; ++i) sum += hist[i];
    uint32_t tot;
    uint32_t acc = block_excl_scan(sum, &tot, sw);
    for (uint32_t i = i0; i < i1; ++i) {
      const uint32_t c = hist[i];
      my_off[i - i0] = acc;
      k.blk_off[((u64)s << k.l2_bits) + i] = (uint32_t)(out0 + acc);
      hist[i] = acc;  // becomes the cursor
      acc += c;
    }
  }
  __syncthreads();
  for (uint32_t chunk = 0; chunk < total; chunk += blockDim.x) {
    combine_clear<L>(cb);
    __syncthreads();
    const uint32_t j = chunk + threadIdx.x;
    KT<L> key = j < total ? keyA[out0 + j] : (KT<L>)0;
    const bool ok = key != 0;
    KT<L> val = 0;
    uint32_t seq = 0, p = 0;
    if (ok) {
      val = valA[out0 + j];
      seq = k.seqA[out0 + j];
      p = combine_claim<L>(cb, key, sort_hash<L>(T, key, k.crc_hi, k.mul));
    }
    __syncthreads();
    combine_values<L>(cb, ok, p, val, seq, k.op);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kSlots; i += blockDim.x) {
      const KT<L> kk = cb.key[i];
      if (kk == 0) continue;
      const uint32_t u = sort_hash<L>(T, kk, k.crc_hi, k.mul);
      const uint32_t q = atomicAdd(&hist[top_bits(u, k.nb_bits) & mask2], 1u);
      keyB[out0 + q] = kk;
      valB[out0 + q] = cb.val[i];
      k.seqB[out0 + q] = cb.seq[i];
    }
    __syncthreads();
  }
  {
    const uint32_t per = (nl2 + blockDim.x - 1) / blockDim.x;
    const uint32_t i0 = std::min(nl2, threadIdx.x * per), i1 = std::min(nl2, i0 + per);
    for (uint32_t i = i0; i < i1; ++i) k.blk_cnt[((u64)s << k.l2_bits) + i] = hist[i] - my_off[i - i0];
  }
}

// ------------------------------------------------------------- stage C

template <int L>
struct BlockLds {
  KT<L> key[kEMax];
  KT<L> val[kEMax];
  uint32_t seq[kEMax];
  uint32_t u[kEMax];
  uint16_t ix[kEMax];
};

template <int L>
__device__ __forceinline__ bool item_less(const BlockLds<L> &b, uint32_t x, uint32_t y) {
  if (b.u[x] != b.u[y]) return b.u[x] < b.u[y];
  if (b.key[x] != b.key[y]) return b.key[x] < b.key[y];
  return b.seq[x] < b.seq[y];
}

// Sorts ix[0..cnt) by an ascending-only bitonic network over the next power
// of two; positions >= cnt act as +infinity and are never touched.
template <int L>
__device__ void lds_bitonic(BlockLds<L> &b, uint32_t cnt) {
  uint32_t P = 1;
  while (P < cnt) P <<= 1;
  for (uint32_t kk = 2; kk <= P; kk <<= 1) {
    for (uint32_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
      const uint32_t half = kk >> 1, blk = t / half, r = t % half;
      const uint32_t i = blk * kk + r, j = blk * kk + kk - 1 - r;
      if (j < cnt && item_less<L>(b, b.ix[j], b.ix[i])) {
        const uint16_t x = b.ix[i];
        b.ix[i] = b.ix[j];
        b.ix[j] = x;
      }
    }
    __syncthreads();
    for (uint32_t jj = kk >> 2; jj >= 1; jj >>= 1) {
      for (uint32_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
        const uint32_t i = 2 * jj * (t / jj) + (t % jj), j = i + jj;
        if (j < cnt && item_less<L>(b, b.ix[j], b.ix[i])) {
          const uint16_t x = b.ix[i];
          b.ix[i] = b.ix[j];
          b.ix[j] = x;
        }
      }
      __syncthreads();
    }
  }
}

// Per-wavefront LDS of the common case: a block of at most kEW elements.
template <int L>
struct WaveLds {
  KT<L> key[kEW];
  KT<L> val[kEW];
  uint32_t seq[kEW];
  uint32_t u[kEW];
  uint16_t ix[kEW];
};

template <int L>
__device__ __forceinline__ bool witem_less(const WaveLds<L> &b, uint32_t x, uint32_t y) {
  if (b.u[x] != b.u[y]) return b.u[x] < b.u[y];
  if (b.key[x] != b.key[y]) return b.key[x] < b.key[y];
  return b.seq[x] < b.seq[y];
}

__device__ __forceinline__ long long wave_max(long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const long long t = __shfl_xor(v, o, 64);
    v = v > t ? v : t;
  }
  return v;
}

// One wavefront per block (4 per workgroup, no workgroup barrier after the
// CRC tables): the block's elements are sorted by a bitonic network in the
// wavefront's LDS, equal keys reduced to their run end, and the carry map
// computed.  Larger blocks are listed for the workgroup and global paths.
template <int L>
__global__ void __launch_bounds__(256) k_bm_block_wave(BmK k) {
  __shared__ uint32_t T[8][256];
  __shared__ WaveLds<L> wl[4];
  if (k.ctl->full) return;
  crc_tables_build(T);
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  WaveLds<L> &b = wl[wv];
  KT<L> *keyB = (KT<L> *)k.keyB;
  KT<L> *valB = (KT<L> *)k.valB;
  const uint32_t B = 1u << k.log2b;
  for (u64 blk = (u64)blockIdx.x * 4 + wv; blk < k.nblocks; blk += (u64)gridDim.x * 4) {
    const uint32_t off = k.blk_off[blk], cnt = k.blk_cnt[blk];
    if (cnt > kEW) {
      if (lane == 0) {
        if (cnt > kEMax)
          k.big_list[atomicAdd(&k.ctl->big_blocks, 1u)] = (uint32_t)blk;
        else
          k.mid_list[atomicAdd(&k.ctl->mid_blocks, 1u)] = (uint32_t)blk;
      }
      continue;
    }
    for (uint32_t i = lane; i < cnt; i += 64) {
      b.key[i] = keyB[(u64)off + i];
      b.val[i] = valB[(u64)off + i];
      b.seq[i] = k.seqB[(u64)off + i];
      b.u[i] = sort_hash<L>(T, b.key[i], k.crc_hi, k.mul);
      b.ix[i] = (uint16_t)i;
    }
    wave_sync();
    uint32_t P = 1;
    while (P < cnt) P <<= 1;
    for (uint32_t kk = 2; kk <= P; kk <<= 1) {
      for (uint32_t t = lane; t < P / 2; t += 64) {
        const uint32_t half = kk >> 1, bl = t / half, r = t % half;
        const uint32_t i = bl * kk + r, j = bl * kk + kk - 1 - r;
        if (j < cnt && witem_less<L>(b, b.ix[j], b.ix[i])) {
          const uint16_t x = b.ix[i];
          b.ix[i] = b.ix[j];
          b.ix[j] = x;
        }
      }
      wave_sync();
      for (uint32_t jj = kk >> 2; jj >= 1; jj >>= 1) {
        for (uint32_t t = lane; t < P / 2; t += 64) {
          const uint32_t i = 2 * jj * (t / jj) + (t % jj), j = i + jj;
          if (j < cnt && witem_less<L>(b, b.ix[j], b.ix[i])) {
            const uint16_t x = b.ix[i];
            b.ix[i] = b.ix[j];
            b.ix[j] = x;
          }
        }
        wave_sync();
      }
    }
    // run ends of equal keys are kept; 4 consecutive sorted positions per lane
    uint32_t keep = 0;
    KT<L> kv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t r = lane * 4 + q;
      if (r < cnt && (r + 1 == cnt || b.key[b.ix[r + 1]] != b.key[b.ix[r]])) {
        keep |= 1u << q;
        KT<L> v = b.val[b.ix[r]];
        if (k.op == 1)
          for (uint32_t r2 = r; r2 > 0 && b.key[b.ix[r2 - 1]] == b.key[b.ix[r]]; --r2) v += b.val[b.ix[r2 - 1]];
        kv[q] = v;
      }
    }
    const uint32_t mine = (uint32_t)__popc(keep);
    const uint32_t incl = wave_incl_scan(mine);
    const uint32_t m = __shfl(incl, 63, 64);
    uint32_t rank = incl - mine;
    long long qmax = LLONG_MIN;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!(keep >> q & 1u)) continue;
      const uint32_t x = b.ix[lane * 4 + q];
      const long long qq = (long long)top_bits(b.u[x], k.log2c) - (long long)rank;
      qmax = qmax > qq ? qmax : qq;
      keyB[(u64)off + rank] = b.key[x];
      valB[(u64)off + rank] = kv[q];
      k.seqB[(u64)off + rank] = b.u[x];  // the hash, for the placement
      ++rank;
    }
    const long long mx = wave_max(qmax);
    if (lane == 0) {
      k.blk_cnt[blk] = m;
      const long long s0 = (long long)(blk << k.log2b);
      const long long a = m ? (long long)m + mx - s0 - (long long)B : 0;
      k.car_a[blk] = a > 0 ? a : 0;
      k.car_d[blk] = (long long)m - (long long)B;
    }
    wave_sync();
  }
}

// Blocks of kEW < elements <= kEMax: one workgroup each, from the list.
template <int L>
__global__ void __launch_bounds__(256) k_bm_block(BmK k) {
  __shared__ uint32_t T[8][256];
  __shared__ BlockLds<L> b;
  __shared__ uint32_t sw[17];
  __shared__ long long sm[17];
  if (k.ctl->full) return;
  crc_tables_build(T);
  KT<L> *keyB = (KT<L> *)k.keyB;
  KT<L> *valB = (KT<L> *)k.valB;
  const uint32_t B = 1u << k.log2b;
  const uint32_t nmid = k.ctl->mid_blocks;
  for (uint32_t mi = blockIdx.x; mi < nmid; mi += gridDim.x) {
    const u64 blk = k.mid_list[mi];
    const uint32_t off = k.blk_off[blk], cnt = k.blk_cnt[blk];
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
      b.key[i] = keyB[(u64)off + i];
      b.val[i] = valB[(u64)off + i];
      b.seq[i] = k.seqB[(u64)off + i];
      b.u[i] = sort_hash<L>(T, b.key[i], k.crc_hi, k.mul);
      b.ix[i] = (uint16_t)i;
    }
    __syncthreads();
    lds_bitonic<L>(b, cnt);
    // run ends of equal keys are kept; 4 sorted positions per thread
    const u64 s0 = blk << k.log2b;
    uint32_t keep = 0;
    KT<L> kv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t r = threadIdx.x * 4 + q;
      if (r < cnt && (r + 1 == cnt || b.key[b.ix[r + 1]] != b.key[b.ix[r]])) {
        keep |= 1u << q;
        KT<L> v = b.val[b.ix[r]];
        if (k.op == 1)
          for (uint32_t r2 = r; r2 > 0 && b.key[b.ix[r2 - 1]] == b.key[b.ix[r]]; --r2) v += b.val[b.ix[r2 - 1]];
        kv[q] = v;
      }
    }
    uint32_t m;
    const uint32_t base = block_excl_scan((uint32_t)__popc(keep), &m, sw);
    long long qmax = LLONG_MIN;
    uint32_t rank = base;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!(keep >> q & 1u)) continue;
      const uint32_t x = b.ix[threadIdx.x * 4 + q];
      const long long pos = (long long)top_bits(b.u[x], k.log2c);
      const long long qq = pos - (long long)rank;
      qmax = qmax > qq ? qmax : qq;
      keyB[(u64)off + rank] = b.key[x];
      valB[(u64)off + rank] = kv[q];
      k.seqB[(u64)off + rank] = b.u[x];  // the hash, for the placement
      ++rank;
    }
    long long mx;
    (void)block_incl_max(qmax, &mx, sm);
    if (threadIdx.x == 0) {
      k.blk_cnt[blk] = m;
      const long long a = m ? (long long)m + mx - (long long)s0 - (long long)B : 0;
      k.car_a[blk] = a > 0 ? a : 0;
      k.car_d[blk] = (long long)m - (long long)B;
    }
    __syncthreads();
  }
}

// Blocks with more than kEMax elements: one workgroup sorts the block's
// range in global memory (the hash of each element kept in the stage-A
// sequence array at the same index), then keeps the run ends.
template <int L>
__device__ __forceinline__ bool g_less(const BmK &k, const uint32_t *u, const KT<L> *key, const uint32_t *seq,
                                       u64 x, u64 y) {
  if (u[x] != u[y]) return u[x] < u[y];
  if (key[x] != key[y]) return key[x] < key[y];
  return seq[x] < seq[y];
}

template <int L>
__global__ void __launch_bounds__(256) k_bm_big_block(BmK k) {
  __shared__ uint32_t T[8][256];
  __shared__ uint32_t sw[17];
  __shared__ long long sm[17];
  __shared__ KT<L> carry_v;
  if (k.ctl->full) return;
  crc_tables_build(T);
  KT<L> *keyB = (KT<L> *)k.keyB;
  KT<L> *valB = (KT<L> *)k.valB;
  uint32_t *uu = k.seqA;
  const uint32_t B = 1u << k.log2b;
  const uint32_t nbig = k.ctl->big_blocks;
  for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
    const u64 blk = k.big_list[bi];
    const u64 off = k.blk_off[blk];
    const uint32_t cnt = k.blk_cnt[blk];
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) uu[off + i] = sort_hash<L>(T, keyB[off + i], k.crc_hi, k.mul);
    __syncthreads();
    u64 P = 1;
    while (P < cnt) P <<= 1;
    auto cswap = [&](u64 i, u64 j) {
      if (j < cnt && g_less<L>(k, uu, keyB, k.seqB, off + j, off + i)) {
        const u64 a = off + i, c = off + j;
        const uint32_t tu = uu[a]; uu[a] = uu[c]; uu[c] = tu;
        const KT<L> tk = keyB[a]; keyB[a] = keyB[c]; keyB[c] = tk;
        const KT<L> tv = valB[a]; valB[a] = valB[c]; valB[c] = tv;
        const uint32_t ts = k.seqB[a]; k.seqB[a] = k.seqB[c]; k.seqB[c] = ts;
      }
    };
    for (u64 kk = 2; kk <= P; kk <<= 1) {
      for (u64 t = threadIdx.x; t < P / 2; t += blockDim.x) {
        const u64 half = kk >> 1, bl = t / half, r = t % half;
        cswap(bl * kk + r, bl * kk + kk - 1 - r);
      }
      __syncthreads();
      for (u64 jj = kk >> 2; jj >= 1; jj >>= 1) {
        for (u64 t = threadIdx.x; t < P / 2; t += blockDim.x) {
          const u64 i = 2 * jj * (t / jj) + (t % jj);
          cswap(i, i + jj);
        }
        __syncthreads();
      }
    }
    // keep run ends, chunk by chunk; with add a run's sum is carried across
    // chunks (segmented scan in LDS over each chunk)
    __shared__ KT<L> sv[256];
    __shared__ uint32_t shd[256];
    if (threadIdx.x == 0) carry_v = 0;
    __syncthreads();
    const u64 s0 = blk << k.log2b;
    uint32_t out = 0;
    long long qmax = LLONG_MIN;
    for (uint32_t c0 = 0; c0 < cnt; c0 += blockDim.x) {
      const uint32_t r = c0 + threadIdx.x;
      const bool in = r < cnt;
      KT<L> key = 0, v = 0;
      uint32_t u = 0;
      bool head = false, end = false;
      if (in) {
        key = keyB[off + r];
        v = valB[off + r];
        u = uu[off + r];
        head = r == 0 || keyB[off + r - 1] != key;
        end = r + 1 == cnt || keyB[off + r + 1] != key;
      }
      __syncthreads();  // every read of this chunk precedes the writes below
      if (k.op == 1) {
        if (threadIdx.x == 0 && !head && in) v += carry_v;
        sv[threadIdx.x] = v;
        shd[threadIdx.x] = head ? 1u : 0u;
        __syncthreads();
        for (uint32_t o = 1; o < 256; o <<= 1) {
          KT<L> add = 0;
          uint32_t hh = 0;
          if (threadIdx.x >= o) {
            add = sv[threadIdx.x - o];
            hh = shd[threadIdx.x - o];
          }
          __syncthreads();
          if (threadIdx.x >= o && !shd[threadIdx.x]) {
            sv[threadIdx.x] += add;
            shd[threadIdx.x] = hh;
          }
          __syncthreads();
        }
        v = sv[threadIdx.x];
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry_v = v;  // partial sum of the chunk's last run
      }
      uint32_t nk;
      const uint32_t rank = out + block_excl_scan(end ? 1u : 0u, &nk, sw);
      if (end) {
        const long long qq = (long long)top_bits(u, k.log2c) - (long long)rank;
        qmax = qmax > qq ? qmax : qq;
        keyB[off + rank] = key;
        valB[off + rank] = v;
        k.seqB[off + rank] = u;
      }
      out += nk;
      __syncthreads();
    }
    long long mx;
    (void)block_incl_max(qmax, &mx, sm);
    if (threadIdx.x == 0) {
      k.blk_cnt[blk] = out;
      const long long a = out ? (long long)out + mx - (long long)s0 - (long long)B : 0;
      k.car_a[blk] = a > 0 ? a : 0;
      k.car_d[blk] = (long long)out - (long long)B;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------- stage D

__device__ __forceinline__ Carry load_carry(const BmK &k, u64 b) {
  Carry c;
  c.a = k.car_a[b];
  c.d = k.car_d[b];
  return c;
}

// Inclusive scan of carry maps over the workgroup (256 threads) in order.
__device__ __forceinline__ Carry block_scan_carry(Carry v, Carry *sc) {
  sc[threadIdx.x] = v;
  __syncthreads();
  for (uint32_t o = 1; o < blockDim.x; o <<= 1) {
    Carry left{0, 0};
    const bool has = threadIdx.x >= o;
    if (has) left = sc[threadIdx.x - o];
    __syncthreads();
    if (has) {
      v = then(left, v);
      sc[threadIdx.x] = v;
    }
    __syncthreads();
  }
  return v;
}

__global__ void __launch_bounds__(256) k_bm_scan_reduce(BmK k) {
  __shared__ Carry sc[256];
  const u64 b0 = (u64)blockIdx.x * kScanTile + (u64)threadIdx.x * kScanPer;
  Carry acc{0, 0};
  for (uint32_t i = 0; i < kScanPer; ++i)
    if (b0 + i < k.nblocks) acc = then(acc, load_carry(k, b0 + i));
  acc = block_scan_carry(acc, sc);
  if (threadIdx.x == blockDim.x - 1) {
    k.tile_a[blockIdx.x] = acc.a;
    k.tile_d[blockIdx.x] = acc.d;
  }
}

// One workgroup: exclusive prefix of the tile maps (in place), the totals,
// the full check and the counts.
__global__ void __launch_bounds__(256) k_bm_scan_top(BmK k) {
  __shared__ Carry sc[256];
  __shared__ Carry run;
  if (threadIdx.x == 0) run = Carry{0, 0};
  __syncthreads();
  for (u64 t0 = 0; t0 < k.ntiles; t0 += blockDim.x) {
    const u64 t = t0 + threadIdx.x;
    Carry v{0, 0};
    if (t < k.ntiles) v = Carry{k.tile_a[t], k.tile_d[t]};
    const Carry incl = block_scan_carry(v, sc);
    const Carry before = run;
    Carry ex{0, 0};
    if (threadIdx.x > 0) ex = sc[threadIdx.x - 1];
    if (t < k.ntiles) {
      const Carry p = threadIdx.x > 0 ? then(before, ex) : before;
      k.tile_a[t] = p.a;
      k.tile_d[t] = p.d;
    }
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) run = then(before, incl);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // all blocks: carry out of the last block, and the distinct total
    const long long distinct = run.d + (long long)k.c;
    const long long wrapped = run.a > run.d ? run.a : run.d;
    k.ctl->distinct = (unsigned long long)distinct;
    k.ctl->wrapped = (unsigned long long)(wrapped > 0 ? wrapped : 0);
    if (k.ctl->full) {
      // an earlier stage stopped
    } else if (distinct > (long long)k.c) {
      k.ctl->full = 1;
      atomicOr(&k.st->err, kErrFull);
    } else {
      add64(&k.st->slot[0].used, (u64)distinct);
      add64(&k.st->slot[0].live, (u64)distinct);
    }
  }
}

__global__ void __launch_bounds__(256) k_bm_scan_down(BmK k) {
  __shared__ Carry sc[256];
  const u64 b0 = (u64)blockIdx.x * kScanTile + (u64)threadIdx.x * kScanPer;
  Carry mine{0, 0};
  for (uint32_t i = 0; i < kScanPer; ++i)
    if (b0 + i < k.nblocks) mine = then(mine, load_carry(k, b0 + i));
  const Carry incl = block_scan_carry(mine, sc);
  (void)incl;
  Carry run = Carry{k.tile_a[blockIdx.x], k.tile_d[blockIdx.x]};
  if (threadIdx.x > 0) run = then(run, sc[threadIdx.x - 1]);
  for (uint32_t i = 0; i < kScanPer; ++i) {
    const u64 b = b0 + i;
    if (b >= k.nblocks) break;
    const long long cin = run.a > run.d ? run.a : run.d;  // the map applied to 0
    k.cin[b] = cin > 0 ? cin : 0;
    run = then(run, load_carry(k, b));
  }
}

// ------------------------------------------------------------- stage E

template <int L>
__device__ __forceinline__ void put_cell(void *cells, u64 p, KT<L> key, KT<L> val) {
  if (L == 0) {
    ((u64 *)cells)[p] = (u64)key | ((u64)val << 32);
  } else {
    u64x2 w;
    w.x = (u64)key;
    w.y = (u64)val;
    ((u64x2 *)cells)[p] = w;
  }
}

// One wavefront per block: element r of the block (in order) goes to
// p = r + max(s + c_in, max_{l<=r}(pos_l - l)); cells of the block itself
// go through an LDS image written once from cell s + min(c_in, B) on.
template <int L>
__global__ void __launch_bounds__(256) k_bm_place(BmK k) {
  __shared__ KT<L> ik[4][256];
  __shared__ KT<L> iv[4][256];
  if (k.ctl->full) return;
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const KT<L> *keyB = (const KT<L> *)k.keyB;
  const KT<L> *valB = (const KT<L> *)k.valB;
  KT<L> *wk = (KT<L> *)k.keyA;
  KT<L> *wvv = (KT<L> *)k.valA;
  const uint32_t B = 1u << k.log2b;
  for (u64 blk = (u64)blockIdx.x * 4 + wv; blk < k.nblocks; blk += (u64)gridDim.x * 4) {
    const u64 s0 = blk << k.log2b;
    const long long cin = k.cin[blk];
    const uint32_t off = k.blk_off[blk], m = k.blk_cnt[blk];
    for (uint32_t i = lane; i < B; i += 64) {
      ik[wv][i] = 0;
      iv[wv][i] = 0;
    }
    wave_sync();
    const long long start = (long long)s0 + cin;
    long long carry_mx = LLONG_MIN;
    for (uint32_t c0 = 0; c0 < m; c0 += 64) {
      const uint32_t r = c0 + lane;
      long long mx = r < m ? (long long)top_bits(k.seqB[(u64)off + r], k.log2c) - (long long)r : LLONG_MIN;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const long long t = __shfl_up(mx, o, 64);
        if (lane >= (uint32_t)o) mx = mx > t ? mx : t;
      }
      mx = mx > carry_mx ? mx : carry_mx;
      if (r < m) {
        const long long p = (long long)r + (mx > start ? mx : start);
        const KT<L> key = keyB[(u64)off + r], val = valB[(u64)off + r];
        if (p < (long long)(s0 + B)) {
          ik[wv][p - (long long)s0] = key;
          iv[wv][p - (long long)s0] = val;
        } else if (p < (long long)k.c) {  // an element that runs into a later block
          put_cell<L>(k.cells, (u64)p, key, val);
        } else if (p - (long long)k.c < (long long)k.cap_items) {  // wrapped: listed in order
          wk[p - (long long)k.c] = key;
          wvv[p - (long long)k.c] = val;
        }
      }
      carry_mx = __shfl(mx, 63, 64);
    }
    wave_sync();
    const uint32_t first = cin < (long long)B ? (uint32_t)cin : B;
    for (uint32_t i = first + lane; i < B; i += 64) put_cell<L>(k.cells, s0 + i, ik[wv][i], iv[wv][i]);
    wave_sync();
  }
}

// ------------------------------------------------------------- stage F

template <int L>
__global__ void __launch_bounds__(256) k_bm_wrap(BmK k) {
  __shared__ uint32_t sw[17];
  if (k.ctl->full) return;
  const u64 W = k.ctl->wrapped;
  const KT<L> *wk = (const KT<L> *)k.keyA;
  const KT<L> *wv = (const KT<L> *)k.valA;
  u64 placed = 0;
  for (u64 base = 0; placed < W && base < k.c; base += blockDim.x) {
    const u64 cell = base + threadIdx.x;
    bool empty = false;
    if (cell < k.c) empty = (L == 0 ? (((const u64 *)k.cells)[cell] & 0xFFFFFFFFull) : ((const u64 *)k.cells)[2 * cell]) == 0;
    uint32_t tot;
    const uint32_t rank = block_excl_scan(empty ? 1u : 0u, &tot, sw);
    if (empty && placed + rank < W && placed + rank < k.cap_items) {
      const u64 j = placed + rank;
      if (L == 0) {
        ((u64 *)k.cells)[cell] = (u64)wk[j] | ((u64)wv[j] << 32);
      } else {
        u64x2 w;
        w.x = (u64)wk[j];
        w.y = (u64)wv[j];
        ((u64x2 *)k.cells)[cell] = w;
      }
    }
    placed += tot;
  }
}

// ------------------------------------------------------------- host

struct Geometry {
  uint32_t log2b, nb_bits, l1_bits, l2_bits, L1, GA;
  uint64_t nblocks, per, ntiles;
};

Geometry geometry(uint64_t ntot, uint32_t log2c) {
  Geometry g{};
  g.log2b = std::min<uint32_t>(8, log2c);
  g.nb_bits = log2c - g.log2b;
  g.l1_bits = std::min<uint32_t>(g.nb_bits, std::max<uint32_t>(8, g.nb_bits > 11 ? g.nb_bits - 11 : 0));
  g.l2_bits = g.nb_bits - g.l1_bits;
  g.L1 = 1u << g.l1_bits;
  g.nblocks = 1ull << g.nb_bits;
  u64 per = (ntot + kGAMax - 1) / kGAMax;
  per = std::max<u64>(4 * kTileA, (per + kTileA - 1) / kTileA * kTileA);
  g.per = per;
  g.GA = (uint32_t)std::max<u64>(1, (ntot + per - 1) / per);
  g.ntiles = (g.nblocks + kScanTile - 1) / kScanTile;
  return g;
}

struct Carve {
  unsigned char *p;
  size_t used = 0;
  template <typename P>
  void take(P *&out, size_t bytes) {
    out = p ? (P *)(p + used) : nullptr;
    used += (bytes + 255) & ~(size_t)255;
  }
};

// Lays the scratch block out (k == nullptr: only sizes it).
void carve_all(Carve &cv, uint64_t N, const Geometry &g, uint32_t layout, BmK &k) {
  const size_t kb = layout == 0 ? 4 : 8;
  N = std::max<uint64_t>(N, 1);
  cv.take(k.ctl, sizeof(BulkMergeCtl));
  cv.take(k.keyA, N * kb);
  cv.take(k.valA, N * kb);
  cv.take(k.seqA, N * 4);
  cv.take(k.keyB, N * kb);
  cv.take(k.valB, N * kb);
  cv.take(k.seqB, N * 4);
  cv.take(k.mcnt, (size_t)g.L1 * g.GA * 4);
  cv.take(k.moff, (size_t)g.L1 * g.GA * 4);
  cv.take(k.l1_off, ((size_t)g.L1 + 1) * 4);
  cv.take(k.blk_off, g.nblocks * 4);
  cv.take(k.blk_cnt, g.nblocks * 4);
  cv.take(k.big_list, g.nblocks * 4);
  cv.take(k.mid_list, g.nblocks * 4);
  cv.take(k.car_a, g.nblocks * 8);
  cv.take(k.car_d, g.nblocks * 8);
  cv.take(k.cin, g.nblocks * 8);
  cv.take(k.tile_a, g.ntiles * 8);
  cv.take(k.tile_d, g.ntiles * 8);
}

}  // namespace

// The fixed scratch of the entry point that allocates nothing
// (lpht_build_noalloc): one array per device, held until the process ends.
// In host code `scratch` names a host-side stand-in, never the device array:
// its device address comes from hipGetSymbolAddress, once per device, with
// that device current, and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kNoAllocDevices];
}  // namespace

hipError_t noalloc_scratch(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= kNoAllocDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_noalloc_ptr[device] = p;
  }
  *out = g_noalloc_ptr[device];
  return hipSuccess;
}

size_t bulk_merge_scratch_bytes(uint64_t inputs, uint64_t max_items, uint32_t log2_new, uint32_t layout) {
  const Geometry g = geometry(inputs, log2_new);
  Carve cv{nullptr};
  BmK k{};
  carve_all(cv, max_items, g, layout, k);
  return cv.used;
}

hipError_t launch_bulk_merge(const BulkMergeArgs &a, hipStream_t s) {
  drop_stale_error();
  if (a.layout > 1 || a.op > 1 || a.log2_new < 6 || a.log2_new > kBulkMaxLog2 || !a.new_cells || !a.scratch ||
      !a.status)
    return hipErrorInvalidValue;
  if (a.n && !a.keys) return hipErrorInvalidValue;
  if (a.old_ncells && !a.old_cells) return hipErrorInvalidValue;
  const uint64_t ntot = a.old_ncells + a.n;
  if (a.max_items >= (1ull << 32) || a.n >= (1ull << 32) - 1) return hipErrorInvalidValue;
  const Geometry g = geometry(ntot, a.log2_new);
  if (g.L1 > kL1Max || (1u << g.l2_bits) > kL2Max || g.GA > kGAMax) return hipErrorInvalidValue;
  BmK k{};
  k.layout = a.layout;
  k.op = a.op;
  k.old_cells = a.old_cells;
  k.cold = a.old_ncells;
  k.keys = a.keys;
  k.vals = a.vals;
  k.n = a.n;
  k.ntot = ntot;
  k.cells = a.new_cells;
  k.log2c = a.log2_new;
  k.log2b = g.log2b;
  k.nb_bits = g.nb_bits;
  k.l1_bits = g.l1_bits;
  k.l2_bits = g.l2_bits;
  k.L1 = g.L1;
  k.GA = g.GA;
  k.c = 1ull << a.log2_new;
  k.cap_items = std::max<uint64_t>(a.max_items, 1);
  k.nblocks = g.nblocks;
  k.per = g.per;
  k.ntiles = g.ntiles;
  k.crc_hi = a.crc_hi;
  k.crc_lo = a.crc_lo;
  k.mul = a.mul;
  k.st = a.status;
  Carve cv{(unsigned char *)a.scratch};
  carve_all(cv, a.max_items, g, a.layout, k);
  hipLaunchKernelGGL(k_bm_init, dim3(1), dim3(64), 0, s, k.ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // one wavefront per block, grid-stride over the blocks
  const uint32_t gwave =
      (uint32_t)std::min<uint64_t>((g.nblocks + 3) / 4, (uint64_t)std::max<uint32_t>(1, a.num_cus) * 16);
#define LPHT_BM(KERN, GRID, THREADS)                                                   \
  do {                                                                                 \
    if (a.layout == 0)                                                                 \
      hipLaunchKernelGGL(KERN<0>, dim3(GRID), dim3(THREADS), 0, s, k);                 \
    else                                                                               \
      hipLaunchKernelGGL(KERN<1>, dim3(GRID), dim3(THREADS), 0, s, k);                 \
    if ((e = hipGetLastError()) != hipSuccess) return e;                               \
  } while (0)
  LPHT_BM(k_bm_count, g.GA, 256);
  hipLaunchKernelGGL(k_bm_scan_rows, dim3(g.L1), dim3(256), 0, s, k);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bm_scan_bins, dim3(1), dim3(1024), 0, s, k);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  LPHT_BM(k_bm_scatter, g.GA, 256);
  LPHT_BM(k_bm_partition, g.L1, 1024);
  LPHT_BM(k_bm_block_wave, gwave, 256);
  LPHT_BM(k_bm_block, 256, 256);
  LPHT_BM(k_bm_big_block, 64, 256);
  hipLaunchKernelGGL(k_bm_scan_reduce, dim3((uint32_t)g.ntiles), dim3(256), 0, s, k);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bm_scan_top, dim3(1), dim3(256), 0, s, k);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bm_scan_down, dim3((uint32_t)g.ntiles), dim3(256), 0, s, k);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  LPHT_BM(k_bm_place, gwave, 256);
  LPHT_BM(k_bm_wrap, 1, 256);
#undef LPHT_BM
  return hipSuccess;
}

}  // namespace lpht
