// Full key space of liblpht (Sec. 5.6): the keys that mark empty and deleted
// cells (0 and 1) are stored in two special slots of the table object
// instead of being refused.  The cell kernels skip such operations; then
//   k_special_list: every lane whose key is 0 or 1 appends its operation's
//     index to a list (one atomic per wavefront);
//   k_special_apply: one workgroup sorts the list and its first lane applies
//     the operations to the two slots in index order -- a valid order of a
//     concurrent call -- writing their flags and found values.
// More than kSpecialList such operations in one call: the workgroup instead
// scans the whole batch in order.

#include <hip/hip_runtime.h>

#include "lpht_device.h"
#include "lpht_special.h"

namespace lpht {

namespace {

template <int L>
__device__ __forceinline__ u64 word_at(const void *a, u64 i) {
  return L == 0 ? (u64)((const uint32_t *)a)[i] : ((const u64 *)a)[i];
}

template <int L>
__global__ void __launch_bounds__(256) k_special_list(const void *keys, uint64_t n, uint32_t *scratch) {
  uint32_t *count = scratch;
  uint32_t *list = scratch + 64;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  // every lane of a wavefront runs the same number of iterations
  const u64 start = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  const u64 iters = (n + stride - 1) / stride;
  for (u64 it = 0; it < iters; ++it) {
    const u64 i = start + it * stride;
    const bool sp = i < n && word_at<L>(keys, i) <= kTomb;
    const u64 m = __ballot(sp);
    if (!m) continue;
    uint32_t base = 0;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t first = __builtin_ctzll(m);
    if (lane == first) base = atomicAdd(count, (uint32_t)__popcll(m));
    base = __shfl(base, first, 64);
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (sp && base + rank < kSpecialList) list[base + rank] = (uint32_t)i;
  }
}

struct Slots {
  u64 p[2], v[2];
};

template <int L>
__device__ void apply_one(Slots &s, OpKind op, uint32_t up, const void *vals, void *vals_out, uint8_t *flags, u64 i,
                          u64 k) {
  const u64 mask = L == 0 ? 0xFFFFFFFFull : ~0ull;
  const u64 d = vals ? word_at<L>(vals, i) : 1;
  uint8_t f = 0;
  u64 out = 0;
  switch (op) {
    case OP_FIND:
      f = s.p[k] ? 1 : 0;
      out = s.p[k] ? s.v[k] : 0;
      break;
    case OP_INSERT:
      if (!s.p[k]) {
        s.p[k] = 1;
        s.v[k] = d & mask;
        f = 1;
      }
      break;
    case OP_UPSERT:
      if (!s.p[k]) {
        s.p[k] = 1;
        s.v[k] = d & mask;
        f = 1;
      } else {
        s.v[k] = (up ? s.v[k] + d : d) & mask;
      }
      break;
    case OP_UPDATE:
      if (s.p[k]) {
        s.v[k] = (up ? s.v[k] + d : d) & mask;
        f = 1;
      }
      break;
    case OP_ERASE:
      if (s.p[k]) {
        s.p[k] = 0;
        s.v[k] = 0;
        f = 1;
      }
      break;
  }
  if (flags) flags[i] = f;
  if (op == OP_FIND && vals_out) {
    if (L == 0)
      ((uint32_t *)vals_out)[i] = (uint32_t)out;
    else
      ((u64 *)vals_out)[i] = out;
  }
}

template <int L>
__global__ void __launch_bounds__(256) k_special_apply(OpKind op, uint32_t up, const void *keys, const void *vals,
                                                       uint64_t n, void *vals_out, uint8_t *flags, SpecialSlots *sp,
                                                       uint32_t *scratch, int clear) {
  __shared__ uint32_t idx[kSpecialList];
  __shared__ uint8_t mark[256];
  const uint32_t total = scratch[0];
  Slots s;
  s.p[0] = clear ? 0 : sp->present[0];
  s.p[1] = clear ? 0 : sp->present[1];
  s.v[0] = clear ? 0 : sp->value[0];
  s.v[1] = clear ? 0 : sp->value[1];
  if (total <= kSpecialList) {
    const uint32_t *list = scratch + 64;
    uint32_t P = 1;
    while (P < total) P <<= 1;
    for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) idx[i] = i < total ? list[i] : 0xFFFFFFFFu;
    __syncthreads();
    // bitonic sort of the indices (padding sorts last)
    for (uint32_t kk = 2; kk <= P; kk <<= 1) {
      for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
        for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) {
          const uint32_t x = i ^ j;
          if (x > i) {
            const bool up_dir = (i & kk) == 0;
            const uint32_t a = idx[i], b = idx[x];
            if ((a > b) == up_dir) {
              idx[i] = b;
              idx[x] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    if (threadIdx.x == 0)
      for (uint32_t q = 0; q < total; ++q) {
        const u64 i = idx[q];
        apply_one<L>(s, op, up, vals, vals_out, flags, i, word_at<L>(keys, i));
      }
  } else {
    // too many for the list: scan the batch in order, 256 at a time
    for (u64 c0 = 0; c0 < n; c0 += blockDim.x) {
      const u64 i = c0 + threadIdx.x;
      mark[threadIdx.x] = (i < n && word_at<L>(keys, i) <= kTomb) ? 1 : 0;
      __syncthreads();
      if (threadIdx.x == 0)
        for (uint32_t q = 0; q < blockDim.x && c0 + q < n; ++q)
          if (mark[q]) apply_one<L>(s, op, up, vals, vals_out, flags, c0 + q, word_at<L>(keys, c0 + q));
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    sp->present[0] = s.p[0];
    sp->present[1] = s.p[1];
    sp->value[0] = s.v[0];
    sp->value[1] = s.v[1];
    scratch[0] = 0;  // ready for the next call
  }
}

}  // namespace

hipError_t launch_special(uint32_t layout, OpKind op, uint32_t up, const void *keys, const void *vals, uint64_t n,
                          void *vals_out, uint8_t *flags, SpecialSlots *sp, uint32_t *scratch, bool clear,
                          hipStream_t s) {
  drop_stale_error();
  if (layout > 1 || !sp || !scratch || (n && !keys)) return hipErrorInvalidValue;
  if (n) {
    u64 blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (layout == 0)
      hipLaunchKernelGGL(k_special_list<0>, dim3((uint32_t)blocks), dim3(256), 0, s, keys, n, scratch);
    else
      hipLaunchKernelGGL(k_special_list<1>, dim3((uint32_t)blocks), dim3(256), 0, s, keys, n, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (layout == 0)
    hipLaunchKernelGGL(k_special_apply<0>, dim3(1), dim3(256), 0, s, op, up, keys, vals, n, vals_out, flags, sp,
                       scratch, clear ? 1 : 0);
  else
    hipLaunchKernelGGL(k_special_apply<1>, dim3(1), dim3(256), 0, s, op, up, keys, vals, n, vals_out, flags, sp,
                       scratch, clear ? 1 : 0);
  return hipGetLastError();
}

}  // namespace lpht
