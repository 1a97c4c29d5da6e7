// Device-side helpers shared by the gfx950 kernels: wave64 ballots and
// scans, block scans, the hash used by the HISA index, and the
// XCD-aware mapping of workgroups to tiles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hl {

typedef uint32_t u32;
typedef uint64_t u64;

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ u64 lanemask_lt() { return (u64(1) << lane_id()) - 1; }

__device__ __forceinline__ u64 ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int popc(u64 x) { return __popcll(x); }

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T t = __shfl_up(v, d, kWave);
    if (lane_id() >= d) v += t;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Exclusive scan over the NT threads of a block, in thread order.
// `lds` must hold NT/64 elements.  Returns the exclusive prefix and writes
// the block total to `total`.  Contains two barriers: every thread of the
// block must call it.
template <int NT, typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* lds, T& total) {
  const int w = threadIdx.x / kWave;
  T inc = wave_inclusive_scan(v);
  if (lane_id() == kWave - 1) lds[w] = inc;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < NT / kWave; ++k) {
    T s = lds[k];
    if (k < w) before += s;
    all += s;
  }
  __syncthreads();
  total = all;
  return before + inc - v;
}

template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T* lds) {
  const int w = threadIdx.x / kWave;
  v = wave_sum(v);
  if (lane_id() == 0) lds[w] = v;
  __syncthreads();
  T all = 0;
#pragma unroll
  for (int k = 0; k < NT / kWave; ++k) all += lds[k];
  __syncthreads();
  return all;
}

// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X, and
// each XCD has its own L2.  Giving each XCD a contiguous range of tiles
// keeps neighbouring tiles' partial cache lines in one L2.  Any bijection
// is correct; this one only matters for speed.
__device__ __forceinline__ u32 xcd_tile(u32 b, u32 nblocks) {
  const u32 nx = 8;
  u32 x = b % nx, idx = b / nx;
  u32 per = nblocks / nx, rem = nblocks % nx;
  return x * per + (x < rem ? x : rem) + idx;
}

// 32-bit finaliser of MurmurHash3 (Appleby), used to spread join keys.
__device__ __forceinline__ u32 mix32(u32 h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// Range reduction of a 32-bit hash to [0, cap) without a division.
__device__ __forceinline__ u64 slot_of(u32 key, u64 cap) {
  return (u64(mix32(key)) * cap) >> 32;
}

}  // namespace hl
