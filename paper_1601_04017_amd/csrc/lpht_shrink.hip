// Shrinking migration of liblpht (Sec. 5.3.1, "Shrinking").
//
// Halving the capacity s times maps the home position h of a key to h >> s,
// so a source block of 256 * 2^s cells maps onto a target block of 256 cells
// and target blocks are disjoint.  The migration runs in two phases:
//
//   1. k_shrink_local: one wavefront per target block.  It walks its source
//      block and places every live element whose new home lies in its target
//      block by linear probing inside that block, in an LDS image of the 256
//      target cells (LDS compare-and-swap, so the lanes act as one sequential
//      inserter).  Elements whose new home lies in another block (they were
//      displaced across the source block boundary) or whose probe would run
//      past the block's end do not fit; they are compacted to the front of
//      the wavefront's own source block, whose cells it has already read, and
//      their number goes to a per-block counter.  The image, empty cells
//      included, is then written to the target block, so the new table needs
//      no separate initialisation.
//   2. k_shrink_rest: after the kernel boundary (the barrier), the elements
//      that did not fit are inserted concurrently with compare-and-swap on
//      the whole target table, with wrap-around.
//
// Both phases are insertions in some sequential order into an initially empty
// table, so the result satisfies the linear probing invariants and its set of
// occupied cells (and each cluster's key set) equals that of the sequential
// migration; only the order of keys inside clusters may differ.
//
// Small target tables (fewer than 2^kShrinkLocalLog2 cells) have too few
// target blocks to spread the source scan over the device; there every live
// element is inserted concurrently (phase 2 alone, over the whole source).

#include <hip/hip_runtime.h>

#include <algorithm>

#include "lpht_device.h"
#include "lpht_shrink.h"

namespace lpht {

namespace {

constexpr uint32_t kWavesPerBlock = 4;
constexpr uint32_t kChunk = 256;  // source cells per wavefront iteration (4 per lane)

// Source cell `i` as two words (PACKED32: the word and 0).
template <int LAYOUT>
__device__ __forceinline__ u64x2 load_cell(const void *cells, u64 i) {
  if (LAYOUT == 0) {
    u64x2 v;
    v.x = ((const u64 *)cells)[i];
    v.y = 0;
    return v;
  }
  return ((const u64x2 *)cells)[i];
}

template <int LAYOUT>
__device__ __forceinline__ u64 key_word(u64x2 c) {
  return LAYOUT == 0 ? (c.x & 0xFFFFFFFFull) : c.x;
}

// Concurrent insertion of a key known to be absent (a migration moves
// distinct keys): claim the first empty cell from `home` on, with
// wrap-around.  PACKED32 claims the whole word; KV64 claims the key word and
// then stores the value (no reader runs during the migration).  Returns false
// if no empty cell was found in one full turn.
template <int LAYOUT>
__device__ __forceinline__ bool insert_absent(void *cells, u64 mask, u64 home, u64x2 c) {
  u64 p = home;
  for (u64 step = 0; step <= mask; ++step) {
    if (LAYOUT == 0) {
      if (cas64((u64 *)cells + p, kEmpty, c.x) == kEmpty) return true;
    } else {
      if (cas64((u64 *)cells + 2 * p, kEmpty, c.x) == kEmpty) {
        ((u64 *)cells)[2 * p + 1] = c.y;
        return true;
      }
    }
    p = (p + 1) & mask;
  }
  return false;
}

// Phase 1.  Block b of the grid serves target blocks kWavesPerBlock * b + w,
// one per wavefront w; `counts[j]` receives the number of elements of target
// block j that did not fit, stored at the front of source block j.
template <int LAYOUT>
__global__ void __launch_bounds__(64 * kWavesPerBlock)
    k_shrink_local(void *old_cells, uint32_t log2_old, void *new_cells, uint32_t log2_new,
                   uint32_t crc_hi, uint32_t crc_lo, u64 mul, uint32_t *counts, DevStatus *st) {
  __shared__ uint32_t T[8][256];
  __shared__ u64 s_key[kWavesPerBlock][kShrinkBlock];  // PACKED32: whole cell words
  __shared__ u64 s_val[LAYOUT == 0 ? 1 : kWavesPerBlock][LAYOUT == 0 ? 1 : kShrinkBlock];
  __shared__ long long s_acc[2];
  __shared__ uint32_t s_err;
  crc_tables_build(T);

  const uint32_t lane = threadIdx.x & 63;
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t sh = log2_old - log2_new;
  const u64 nblocks = 1ull << (log2_new - 8);
  const u64 j = (u64)blockIdx.x * kWavesPerBlock + w;
  long long placed = 0;

  if (j < nblocks) {
    u64 *sk = s_key[w];
    u64 *sv = s_val[LAYOUT == 0 ? 0 : w];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      sk[lane + 64 * k] = kEmpty;
      if (LAYOUT == 1) sv[lane + 64 * k] = 0;
    }
    wave_sync();

    const u64 src = j << (8 + sh);            // first source cell
    const u64 src_end = src + (256ull << sh);
    u64 out = src;                            // next slot for an element that did not fit
    u64x2 cur[4], nxt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) cur[k] = load_cell<LAYOUT>(old_cells, src + lane + 64 * k);
    for (u64 c = src; c < src_end; c += kChunk) {
      // the next chunk is read ahead; the compacted writes below land before
      // c + kChunk, in cells that are already read
      if (c + kChunk < src_end) {
#pragma unroll
        for (int k = 0; k < 4; ++k) nxt[k] = load_cell<LAYOUT>(old_cells, c + kChunk + lane + 64 * k);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const u64 key = key_word<LAYOUT>(cur[k]);
        bool spill = false;
        if (key != kEmpty && key != kTomb) {
          const u64 h = home_of<LAYOUT>(T, key, crc_hi, crc_lo, mul, log2_new);
          if ((h >> 8) != j) {
            spill = true;
          } else {
            uint32_t p = (uint32_t)h & (kShrinkBlock - 1);
            for (;;) {
              const u64 prev = atomicCAS(&sk[p], (u64)kEmpty, cur[k].x);
              if (prev == kEmpty) {
                if (LAYOUT == 1) sv[p] = cur[k].y;
                ++placed;
                break;
              }
              if (++p == kShrinkBlock) {
                spill = true;
                break;
              }
            }
          }
        }
        const u64 m = __ballot(spill);
        if (m) {
          const uint32_t rank =
              __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
          if (spill) {
            if (LAYOUT == 0)
              ((u64 *)old_cells)[out + rank] = cur[k].x;
            else
              ((u64x2 *)old_cells)[out + rank] = cur[k];
          }
          out += (u64)__popcll(m);
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) cur[k] = nxt[k];
    }
    wave_sync();
    const u64 dst = j << 8;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t i = lane + 64 * k;
      if (LAYOUT == 0) {
        ((u64 *)new_cells)[dst + i] = sk[i];
      } else {
        u64x2 v;
        v.x = sk[i];
        v.y = sv[i];
        ((u64x2 *)new_cells)[dst + i] = v;
      }
    }
    if (lane == 0) counts[j] = (uint32_t)(out - src);
  }
  flush_counts(st, placed, placed, 0u, s_acc, &s_err);
}

// Phase 2.  ALL = false: thread r inserts the counts[r] elements stored at
// the front of source block r.  ALL = true: every live element of the source
// table is inserted (grid-stride over its cells).
template <int LAYOUT, bool ALL>
__global__ void __launch_bounds__(256)
    k_shrink_rest(const void *old_cells, uint32_t log2_old, void *new_cells, uint32_t log2_new,
                  uint32_t crc_hi, uint32_t crc_lo, u64 mul, const uint32_t *counts, DevStatus *st) {
  __shared__ uint32_t T[8][256];
  __shared__ long long s_acc[2];
  __shared__ uint32_t s_err;
  crc_tables_build(T);

  const u64 mask = (1ull << log2_new) - 1;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  long long placed = 0;
  uint32_t err = 0;
  auto move = [&](u64x2 c) {
    const u64 key = key_word<LAYOUT>(c);
    if (key == kEmpty || key == kTomb) return;
    const u64 h = home_of<LAYOUT>(T, key, crc_hi, crc_lo, mul, log2_new);
    if (insert_absent<LAYOUT>(new_cells, mask, h, c))
      ++placed;
    else
      err |= kErrFull;
  };
  if (ALL) {
    const u64 n = 1ull << log2_old;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
      move(load_cell<LAYOUT>(old_cells, i));
  } else {
    const uint32_t sh = log2_old - log2_new;
    const u64 nblocks = 1ull << (log2_new - 8);
    for (u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x; r < nblocks; r += stride) {
      const uint32_t cnt = counts[r];
      const u64 src = r << (8 + sh);
      for (uint32_t i = 0; i < cnt; ++i) move(load_cell<LAYOUT>(old_cells, src + i));
    }
  }
  flush_counts(st, placed, placed, err, s_acc, &s_err);
}

uint32_t capped_grid(u64 items, uint32_t threads, const LaunchCfg &cfg) {
  u64 blocks = (items + threads - 1) / threads;
  const u64 cap = (u64)cfg.num_cus * 16;
  return (uint32_t)std::max<u64>(1, std::min(blocks, cap));
}

}  // namespace

size_t shrink_scratch_bytes(uint32_t log2_old, uint32_t log2_new) {
  if (log2_new >= log2_old || log2_new < kShrinkLocalLog2) return 0;
  return sizeof(uint32_t) << (log2_new - 8);
}

hipError_t launch_shrink(void *old_cells, uint32_t log2_old, void *new_cells, uint32_t log2_new,
                         uint32_t layout, uint32_t crc_hi, uint32_t crc_lo, uint64_t mul, uint32_t *scratch,
                         DevStatus *st, const LaunchCfg &cfg, hipStream_t s) {
  drop_stale_error();
  if (log2_new >= log2_old || log2_old > 40 || layout > 1) return hipErrorInvalidValue;
  if (log2_new >= kShrinkLocalLog2) {
    if (!scratch) return hipErrorInvalidValue;
    const u64 nblocks = 1ull << (log2_new - 8);
    const uint32_t grid = (uint32_t)((nblocks + kWavesPerBlock - 1) / kWavesPerBlock);
    if (layout == 0)
      hipLaunchKernelGGL(k_shrink_local<0>, dim3(grid), dim3(64 * kWavesPerBlock), 0, s, old_cells, log2_old,
                         new_cells, log2_new, crc_hi, crc_lo, (u64)mul, scratch, st);
    else
      hipLaunchKernelGGL(k_shrink_local<1>, dim3(grid), dim3(64 * kWavesPerBlock), 0, s, old_cells, log2_old,
                         new_cells, log2_new, crc_hi, crc_lo, (u64)mul, scratch, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint32_t g2 = capped_grid(nblocks, 256, cfg);
    if (layout == 0)
      hipLaunchKernelGGL((k_shrink_rest<0, false>), dim3(g2), dim3(256), 0, s, old_cells, log2_old, new_cells,
                         log2_new, crc_hi, crc_lo, (u64)mul, scratch, st);
    else
      hipLaunchKernelGGL((k_shrink_rest<1, false>), dim3(g2), dim3(256), 0, s, old_cells, log2_old, new_cells,
                         log2_new, crc_hi, crc_lo, (u64)mul, scratch, st);
    return hipGetLastError();
  }
  hipError_t e = launch_fill_zero(new_cells, (size_t)(layout == 0 ? 8 : 16) << log2_new, cfg, s);
  if (e != hipSuccess) return e;
  const uint32_t g = capped_grid(1ull << log2_old, 256, cfg);
  if (layout == 0)
    hipLaunchKernelGGL((k_shrink_rest<0, true>), dim3(g), dim3(256), 0, s, old_cells, log2_old, new_cells,
                       log2_new, crc_hi, crc_lo, (u64)mul, nullptr, st);
  else
    hipLaunchKernelGGL((k_shrink_rest<1, true>), dim3(g), dim3(256), 0, s, old_cells, log2_old, new_cells,
                       log2_new, crc_hi, crc_lo, (u64)mul, nullptr, st);
  return hipGetLastError();
}

}  // namespace lpht
