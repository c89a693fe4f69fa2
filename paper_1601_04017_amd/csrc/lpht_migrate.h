// Block-parallel cluster migration (Sec. 5.3.1, Lemma 1) by one wavefront
// per block of old cells, shared by the migration kernel (lpht_kernels.hip)
// and the insertion kernel that grows the table while it runs
// (lpht_async.hip).
//
// A wavefront owns old block [d, d + B) and the new range [g d, g (d + B))
// (g = gamma, 1 or 2).  It loads the window [d - H, d + B + H) of old cells
// (H = MIG_HALO) lane-consecutively into registers (the caller prefetches the
// next block's window before working on the current one) and then
//   - stores each window cell's key and value and the image slot of its new
//     home (or empty / tombstone) in LDS;
//   - finds the empty cells with ballots, hence the window range [lo, hi) of
//     the clusters that overlap the block and their starts;
//   - re-inserts each such cluster in old-array order (one lane per cluster;
//     Lemma 1 makes their target ranges disjoint) into an image of the new
//     range that holds 16-bit indices into the window.  The target range of
//     a cluster starting at window cell s begins at image slot g s, and the
//     lane keeps the first 64 of its cells in a register mask, so the first
//     free cell from an element's home is found with one bit scan; only
//     beyond those 64 cells does it probe the image in LDS.  The cells'
//     states are loaded four at a time, ahead of their placement;
//   - streams the owned part of the image out as whole cells.
// Elements of the last cluster that land past the owned range are written by
// the next block's wavefront, which sees that cluster as its incoming one; the
// first block's incoming cluster is the one that wraps around the table end.
// Positions are kept unwrapped (old cell x may be negative for block 0).  A
// cluster longer than the halo (or a table without empty cells) sets
// `overflow`; the caller then redoes the whole move another way.
#pragma once

#include "lpht_device.h"

namespace lpht {

constexpr int MIG_HALO = 128;
constexpr uint16_t kImgEmpty = 0xFFFF;

__host__ __device__ constexpr uint32_t mig_window(uint32_t mb) { return mb + 2 * MIG_HALO; }

// LDS of one wavefront: window keys and values (u64 each; PACKED32 keeps the
// word in the key array), each window cell's state (i16: the new home's image
// slot, below 2 * 1280, or one of the negative codes below), the image (u16
// per new cell) and the list of cluster starts (u16 per start, at most half
// the window).
__host__ __device__ constexpr size_t mig_wave_lds(uint32_t mb, uint32_t layout, uint32_t gamma) {
  return ((size_t)mig_window(mb) * ((layout == 0 ? 8u : 16u) + 2u + 1u) + (size_t)gamma * mig_window(mb) * 2u +
          15) &
         ~(size_t)15;
}
// The scattering form keeps keys and values in registers: cell states, the
// image, the cluster starts and each window cell's new slot (u16).
__host__ __device__ constexpr size_t mig_wave_lds_scatter(uint32_t mb, uint32_t gamma) {
  return ((size_t)mig_window(mb) * (2u + 1u + 2u) + (size_t)gamma * mig_window(mb) * 2u + 15) & ~(size_t)15;
}
constexpr int32_t kCellEmpty = -1, kCellTomb = -2, kCellFar = -3;  // window cell states


// The window of block b (cells t = lane + 64 q, q < Q, of [b B - H, ...)),
// wrapped modulo the old capacity (mask = capacity - 1).  COH: device-coherent
// loads (agent-scope relaxed atomics), for a table that other wavefronts of
// the same launch wrote.
template <int LAYOUT, int Q, bool COH = false>
__device__ __forceinline__ void mig_load_window(u64 (&nk)[Q], u64 (&nv)[Q], const void *old_cells, u64 mask,
                                                u64 b) {
  constexpr uint32_t mb = 64 * Q - 2 * MIG_HALO;
  const uint32_t lane = threadIdx.x & 63;
  const long long wb = (long long)(b * mb) - MIG_HALO;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const u64 x = (u64)(wb + (long long)(lane + 64 * q)) & mask;
    if (LAYOUT == 0) {
      nk[q] = Cells<0>::word<COH>(old_cells, x);
      nv[q] = 0;
    } else {
      const u64x2 c = Cells<1>::cell<COH>(old_cells, x);
      nk[q] = c.x;
      nv[q] = c.y;
    }
  }
}

// Migrates block `blk` from its window (k, v) into the new table of
// 2^(log2_old + g) cells; `base` is the wavefront's mig_wave_lds(B, LAYOUT,
// 2^g) bytes of LDS (SCATTER: mig_wave_lds_scatter(B, 2^g)).  Returns the
// number of elements written.
//   SCATTER: instead of gathering the owned image from keys and values kept
//     in LDS, each lane stores its own elements that landed in the owned range
//     from its registers and the empty owned cells are zeroed (less LDS, more
//     wavefronts where LDS is short); nothing is written after an overflow.
//   COH: the new cells are written with device-coherent stores (agent-scope
//     relaxed atomics), for readers in the same launch.
template <int LAYOUT, int Q, bool SCATTER = false, bool COH = false>
__device__ __forceinline__ long long mig_block(const u64 (&k)[Q], const u64 (&v)[Q], u64 blk, uint32_t log2_old,
                                               uint32_t g, const uint32_t (*T)[256], uint32_t crc_hi, uint32_t crc_lo,
                                               u64 mul, unsigned char *base, void *new_cells, bool &overflow) {
  constexpr int H = MIG_HALO;
  constexpr uint32_t W = 64 * Q;  // window cells
  constexpr uint32_t mb = W - 2 * H;
  static_assert(H % 64 == 0 && mb % 64 == 0, "window of whole lane rows");
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t gamma = 1u << g;  // 1 or 2
  const uint32_t IW = gamma * W;   // image slots
  u64 *wkey = (u64 *)base;  // gather only
  u64 *wval = wkey + W;     // gather, KV64 only
  static_assert(2 * 64 * Q < 32768, "image slots fit the 16-bit cell states");
  int16_t *wnh = (int16_t *)(SCATTER ? base : (unsigned char *)(wkey + (LAYOUT == 0 ? W : 2 * W)));
  uint16_t *img = (uint16_t *)(wnh + W);
  uint16_t *starts = img + IW;        // cluster starts of [lo, hi)
  uint16_t *newpos = starts + W / 2;  // scatter only: image slot each element went to
  const u64 cap = 1ull << log2_old, mask = cap - 1;
  const uint32_t log2_new = log2_old + g;
  long long moved = 0;
  const long long d = (long long)(blk * mb);
  const long long wbase = d - H;  // unwrapped old index of window cell 0
  u64 emp[Q];         // ballot of empty window cells, 64 per word
  uint32_t elem = 0;  // bit q: this lane's cell of row q holds an element
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const uint32_t t = lane + 64 * q;
    const u64 key = LAYOUT == 0 ? (k[q] & 0xFFFFFFFFull) : k[q];
    if (!SCATTER) {
      wkey[t] = k[q];
      if (LAYOUT == 1) wval[t] = v[q];
    }
    emp[q] = __ballot(key == kEmpty);
  }
  for (uint32_t t = lane; t < IW / 2; t += 64) ((uint32_t *)img)[t] = 0xFFFFFFFFu;
  // the window range [lo, hi) of the clusters overlapping the block
  // (cell H - 1 and cell H both non-empty: a cluster comes in from before);
  // every index into emp[] is a constant, so it stays in registers
  int lo = H, hi = H + (int)mb;
  bool skip = false;
  if (!((emp[H / 64 - 1] >> 63) & 1ull) && !(emp[H / 64] & 1ull)) {
    int last = -1;
#pragma unroll
    for (int q = 0; q < H / 64; ++q)
      if (emp[q]) last = 64 * q + 63 - __builtin_clzll(emp[q]);
    if (last < 0) skip = true;
    lo = last + 1;
  }
  if (!((emp[(H + mb) / 64 - 1] >> 63) & 1ull)) {
    int first = -1;
#pragma unroll
    for (int q = Q - 1; q >= 0; --q) {
      if (64 * q < H + (int)mb) break;
      if (emp[q]) first = 64 * q + __builtin_ctzll(emp[q]);
    }
    if (first < 0) skip = true;
    hi = first;
  }
  // each cell's state; only the cells of [lo, hi) are walked, so only their
  // keys are hashed (the halo rows outside it are mostly skipped whole)
  if (!skip) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (64 * q + 63 < lo || 64 * q >= hi) continue;  // the row lies outside [lo, hi)
      const int t = (int)lane + 64 * q;
      const u64 key = LAYOUT == 0 ? (k[q] & 0xFFFFFFFFull) : k[q];
      int32_t rel = key == kEmpty ? kCellEmpty : kCellTomb;
      if (key != kEmpty && key != kTomb && t >= lo && t < hi) {
        // new home, unwrapped consistently with this cell's old position
        const u64 hn = home_of<LAYOUT>(T, key, crc_hi, crc_lo, mul, log2_new);
        const u64 oh = hn >> g;
        const long long x = wbase + (long long)t;
        const u64 delta = ((u64)x - oh) & mask;
        const long long nh = (long long)gamma * (x - (long long)delta) + (long long)(hn & (gamma - 1));
        const long long r = nh - (long long)gamma * wbase;  // image slot of the home
        rel = (r < 0 || r >= (long long)IW) ? kCellFar : (int32_t)r;
        elem |= 1u << q;
      }
      wnh[t] = (int16_t)rel;
    }
  }
  wave_sync();
  if (skip) {
    overflow = true;
  } else {
    // the cluster starts in [lo, hi) (non-empty cells after an empty one),
    // listed in LDS; lanes then take them round-robin, each walking its
    // clusters in old-array order
    uint32_t nstarts = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int t = (int)lane + 64 * q;
      const bool here_empty = (emp[q] >> lane) & 1ull;
      const bool prev_empty =
          lane ? (bool)((emp[q] >> (lane - 1)) & 1ull) : (q == 0 ? true : (bool)(emp[q > 0 ? q - 1 : 0] >> 63));
      const bool st0 = t >= lo && t < hi && !here_empty && prev_empty;
      const u64 m = __ballot(st0);
      if (st0) starts[nstarts + __builtin_popcountll(m & ((1ull << lane) - 1))] = (uint16_t)t;
      nstarts += (uint32_t)__builtin_popcountll(m);
    }
    wave_sync();
    bool bad = false;
    for (uint32_t i = lane; i < nstarts && !bad; i += 64) {
      const int st = starts[i];
      const int tb = (int)gamma * st;  // first image slot of the cluster's target range
      u64 taken = 0;                   // its cells tb .. tb + 63 taken so far
      // places the element of window cell u with state c: 0 placed or a
      // tombstone, 1 the cluster ended, 2 overflow
      auto place = [&](int c, int u) -> int {
        if (c == kCellEmpty) return 1;
        if (c == kCellTomb) return 0;
        if (c < tb) return 2;  // far: its home lies before the window
        int p;
        const int off = c - tb;
        const u64 fr = off < 64 ? ~taken & (~0ull << off) : 0ull;
        if (fr) {
          p = tb + __builtin_ctzll(fr);
        } else {
          p = off < 64 ? tb + 64 : c;
          while (p < (int)IW && img[p] != kImgEmpty) ++p;
        }
        if (p >= (int)IW) return 2;
        if (p - tb < 64) taken |= 1ull << (p - tb);
        img[p] = (uint16_t)u;
        if (SCATTER) newpos[u] = (uint16_t)p;
        return 0;
      };
      // the cells' states are loaded four ahead of their placement
      auto state = [&](int u) -> int { return u < hi ? wnh[u] : kCellEmpty; };
      int c0 = state(st), c1 = state(st + 1), c2 = state(st + 2), c3 = state(st + 3);
      for (int u = st;; u += 4) {
        const int n0 = state(u + 4), n1 = state(u + 5), n2 = state(u + 6), n3 = state(u + 7);
        int r = place(c0, u);
        if (!r) r = place(c1, u + 1);
        if (!r) r = place(c2, u + 2);
        if (!r) r = place(c3, u + 3);
        if (r) {
          bad |= r == 2;
          break;
        }
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
      }
    }
    const u64 dst0 = (u64)d * gamma;
    const uint32_t o0 = gamma * H, n_out = gamma * mb;  // the owned image slots [o0, o0 + n_out)
    auto put = [&](u64 x, u64 kw, u64 vw) {
      if (LAYOUT == 0) {
        if (COH)
          __hip_atomic_store((u64 *)new_cells + x, kw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
          ((u64 *)new_cells)[x] = kw;
      } else if (COH) {
        __hip_atomic_store((u64 *)new_cells + 2 * x, kw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store((u64 *)new_cells + 2 * x + 1, vw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        ((u64x2 *)new_cells)[x] = u64x2{kw, vw};
      }
    };
    if (SCATTER) {
      if (__any(bad)) {
        overflow = true;  // the caller redoes the move; nothing is written
      } else {
        wave_sync();
        // the lane's own elements placed in the owned range, then zeros in
        // the owned cells left empty
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int t = (int)lane + 64 * q;
          if (!((elem >> q) & 1u) || t < lo || t >= hi) continue;
          const uint32_t o = (uint32_t)newpos[t] - o0;  // wraps when below the owned range
          if (o >= n_out) continue;
          put(dst0 + o, k[q], v[q]);
          ++moved;
        }
        for (uint32_t t = lane; t < n_out; t += 64)
          if (img[o0 + t] == kImgEmpty) put(dst0 + t, 0ull, 0ull);
      }
    } else {
      if (bad) overflow = true;
      wave_sync();
      // the owned new cells [g*d, g*(d+B)) = image slots [g*H, g*(H+B))
      for (uint32_t t = lane; t < n_out; t += 64) {
        const uint16_t ix = img[o0 + t];
        const bool e = ix == kImgEmpty;
        const uint32_t j = e ? 0u : ix;
        const u64 kw = wkey[j], vw = LAYOUT == 1 ? wval[j] : 0ull;
        put(dst0 + t, e ? 0ull : kw, e ? 0ull : vw);
        moved += !e;
      }
    }
  }
  wave_sync();
  return moved;
}

}  // namespace lpht
