// Memory-system ceilings for the hash table's access pattern, measured on the
// device the table runs on (gfx950).  These kernels do no table work; the
// benchmark divides the table kernels' rates by them.
//
//   rl_gather     : random aligned loads of `width` bytes (8, 16, 64 or 128)
//                   from a buffer, `per_thread` independent loads per lane
//   rl_cas        : random 64-bit compare-and-swap, device scope
//   rl_add        : random 64-bit fetch-and-add, device scope
//   rl_hot_add    : fetch-and-add on one address by every lane
//   rl_copy       : streaming copy with 16-byte accesses
//
// Random offsets come from a counter-based mix (the SplitMix64 output
// function) of the global lane index and the iteration, so no index array is
// read.  Every kernel folds what it loads into a sink word so the loads are
// not removed.

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned long long u64;
typedef u64 u64x2 __attribute__((ext_vector_type(2)));

namespace {

__device__ __forceinline__ u64 mix64(u64 z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

template <int W, int PER>
__global__ void __launch_bounds__(256) k_gather(const u64 *buf, u64 nunits, u64 seed, u64 *sink) {
  const u64 g = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  const u64 mask = nunits - 1;
  u64 acc = 0;
  constexpr int WORDS = W / 8;
  u64 idx[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) idx[j] = mix64(seed + g * PER + j) & mask;
  if (WORDS == 1) {
    u64 v[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) v[j] = buf[idx[j]];
#pragma unroll
    for (int j = 0; j < PER; ++j) acc ^= v[j];
  } else {
    const u64x2 *b2 = (const u64x2 *)buf;
    u64x2 v[PER][WORDS / 2];
#pragma unroll
    for (int j = 0; j < PER; ++j)
#pragma unroll
      for (int w = 0; w < WORDS / 2; ++w) v[j][w] = b2[idx[j] * (WORDS / 2) + w];
#pragma unroll
    for (int j = 0; j < PER; ++j)
#pragma unroll
      for (int w = 0; w < WORDS / 2; ++w) acc ^= v[j][w].x ^ v[j][w].y;
  }
  if (acc == 0x123456789ull) sink[0] = acc;
}

template <int PER>
__global__ void __launch_bounds__(256) k_cas(u64 *buf, u64 nwords, u64 seed, u64 *sink) {
  const u64 g = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  const u64 mask = nwords - 1;
  u64 acc = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    u64 expected = 0;
    u64 *p = buf + (mix64(seed + g * PER + j) & mask);
    __hip_atomic_compare_exchange_strong(p, &expected, g + 2, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    acc ^= expected;
  }
  if (acc == 0x123456789ull) sink[0] = acc;
}

template <int PER>
__global__ void __launch_bounds__(256) k_add(u64 *buf, u64 nwords, u64 seed, u64 *sink) {
  const u64 g = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  const u64 mask = nwords - 1;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    u64 *p = buf + (mix64(seed + g * PER + j) & mask);
    __hip_atomic_fetch_add(p, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void __launch_bounds__(256) k_hot_add(u64 *word, int per) {
  for (int j = 0; j < per; ++j) __hip_atomic_fetch_add(word, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Streaming copy: a workgroup copies tiles of 256 x COPY_PER 16-byte units;
// each lane issues its COPY_PER loads (coalesced across the workgroup) before
// any store, so many loads are in flight, and stores bypass the caches
// (non-temporal), since nothing reads the destination again.
constexpr int COPY_PER = 8;
__global__ void __launch_bounds__(256) k_copy(const u64x2 *src, u64x2 *dst, u64 n16) {
  const u64 tile = 256ull * COPY_PER;
  const u64 ntiles = n16 / tile;
  for (u64 t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const u64 b = t * tile + threadIdx.x;
    u64x2 v[COPY_PER];
#pragma unroll
    for (int j = 0; j < COPY_PER; ++j) v[j] = __builtin_nontemporal_load(src + b + 256ull * j);
#pragma unroll
    for (int j = 0; j < COPY_PER; ++j) __builtin_nontemporal_store(v[j], dst + b + 256ull * j);
  }
  // the ragged end (fewer than one tile)
  for (u64 i = ntiles * tile + (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += (u64)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

extern "C" {

// Each entry point launches one kernel on `stream` and returns a hipError_t
// value.  `buf` must hold a power-of-two number of `width`-byte units.

int rl_gather(const void *buf, uint64_t bytes, int width, uint64_t lanes, uint64_t seed, void *sink,
              void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const u64 units = bytes / (u64)width;
  if (units == 0 || (units & (units - 1)) || lanes % 256) return (int)hipErrorInvalidValue;
  constexpr int PER = 4;
  const dim3 grid((unsigned)(lanes / 256)), blk(256);
  switch (width) {
    case 8: hipLaunchKernelGGL((k_gather<8, PER>), grid, blk, 0, s, (const u64 *)buf, units, seed, (u64 *)sink); break;
    case 16: hipLaunchKernelGGL((k_gather<16, PER>), grid, blk, 0, s, (const u64 *)buf, units, seed, (u64 *)sink); break;
    case 64: hipLaunchKernelGGL((k_gather<64, PER>), grid, blk, 0, s, (const u64 *)buf, units, seed, (u64 *)sink); break;
    case 128: hipLaunchKernelGGL((k_gather<128, PER>), grid, blk, 0, s, (const u64 *)buf, units, seed, (u64 *)sink); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

int rl_cas(void *buf, uint64_t bytes, uint64_t lanes, uint64_t seed, void *sink, void *stream) {
  const u64 words = bytes / 8;
  if (words == 0 || (words & (words - 1)) || lanes % 256) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL((k_cas<4>), dim3((unsigned)(lanes / 256)), dim3(256), 0, (hipStream_t)stream, (u64 *)buf,
                     words, seed, (u64 *)sink);
  return (int)hipGetLastError();
}

int rl_add(void *buf, uint64_t bytes, uint64_t lanes, uint64_t seed, void *sink, void *stream) {
  const u64 words = bytes / 8;
  if (words == 0 || (words & (words - 1)) || lanes % 256) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL((k_add<4>), dim3((unsigned)(lanes / 256)), dim3(256), 0, (hipStream_t)stream, (u64 *)buf,
                     words, seed, (u64 *)sink);
  return (int)hipGetLastError();
}

int rl_hot_add(void *word, uint64_t lanes, int per_lane, void *stream) {
  if (lanes % 256) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_hot_add, dim3((unsigned)(lanes / 256)), dim3(256), 0, (hipStream_t)stream, (u64 *)word,
                     per_lane);
  return (int)hipGetLastError();
}

int rl_copy(const void *src, void *dst, uint64_t bytes, uint64_t lanes, void *stream) {
  if (bytes % 16 || lanes % 256) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)(lanes / 256)), dim3(256), 0, (hipStream_t)stream,
                     (const u64x2 *)src, (u64x2 *)dst, bytes / 16);
  return (int)hipGetLastError();
}

}  // extern "C"
