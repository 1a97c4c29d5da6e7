// Device-wide exclusive prefix sum: reduce tiles, scan the tile sums
// (recursively), then scan each tile with its offset.  Used for join output
// offsets and for the digit offsets of the radix sort.
#include "device.hpp"
#include "kernels.hpp"

namespace hl {

namespace {

constexpr int kNT = 256;
constexpr int kItems = 8;
constexpr u64 kTile = kNT * kItems;
constexpr u64 kSingleTiles = 4;  // inputs up to this many tiles scan in one block

// Eight consecutive values of in from i (zero past n): two or four 16-byte
// loads when the eight lie inside the array and the address is aligned.
template <typename Tin>
__device__ __forceinline__ void load_items(const Tin* in, u64 i, u64 n, u64 (&v)[kItems]) {
  const Tin* p = in + i;
  if (i + kItems <= n && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
    if constexpr (sizeof(Tin) == 4) {
      const uint4 a = reinterpret_cast<const uint4*>(p)[0];
      const uint4 b = reinterpret_cast<const uint4*>(p)[1];
      v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w;
      v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
    } else {
#pragma unroll
      for (int k = 0; k < kItems / 2; ++k) {
        const ulonglong2 a = reinterpret_cast<const ulonglong2*>(p)[k];
        v[2 * k] = a.x;
        v[2 * k + 1] = a.y;
      }
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < kItems; ++j) v[j] = (i + j < n) ? u64(p[j]) : 0;
}

// Sum of each tile: every thread reads its eight consecutive values with
// load_items (all loads issued before any is added; a conditional add per
// load waited for each load in turn).
template <typename Tin>
__global__ __launch_bounds__(kNT) void scan_reduce_kernel(const Tin* in, u64 n, u64* sums) {
  __shared__ u64 lds[kNT / kWave];
  u64 v[kItems];
  load_items(in, u64(blockIdx.x) * kTile + u64(threadIdx.x) * kItems, n, v);
  u64 s = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) s += v[j];
  s = block_sum<kNT>(s, lds);
  if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

// offsets == nullptr: one block scans `tiles` tiles in turn, from 0.
// Each thread takes kItems consecutive values: a serial scan of its own,
// one block scan of the thread totals, then its outputs written together.
template <typename Tin>
__global__ __launch_bounds__(kNT) void scan_down_kernel(const Tin* in, u64 n, const u64* offsets,
                                                        u64* out, u64* d_total, u32 tiles = 1) {
  __shared__ u64 lds[kNT / kWave];
  u64 carry = offsets ? offsets[blockIdx.x] : 0;
  for (u32 q = 0; q < tiles; ++q) {
    const u64 i0 = (u64(blockIdx.x) + q) * kTile + u64(threadIdx.x) * kItems;
    u64 v[kItems];
    load_items(in, i0, n, v);
    u64 run = 0;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const u64 x = v[j];
      v[j] = run;
      run += x;
    }
    u64 tot;
    const u64 ex = carry + block_exclusive_scan<kNT>(run, lds, tot);
    u64* o = out + i0;
    if (i0 + kItems <= n && (reinterpret_cast<uintptr_t>(o) & 15) == 0) {
#pragma unroll
      for (int k = 0; k < kItems / 2; ++k)
        reinterpret_cast<ulonglong2*>(o)[k] = make_ulonglong2(ex + v[2 * k], ex + v[2 * k + 1]);
    } else {
#pragma unroll
      for (int j = 0; j < kItems; ++j)
        if (i0 + j < n) o[j] = ex + v[j];
    }
    carry += tot;
  }
  if (d_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *d_total = carry;
}

__global__ void set_u64_kernel(u64* p, u64 v) { *p = v; }

u64 tiles_of(u64 n) { return (n + kTile - 1) / kTile; }

template <typename Tin>
hipError_t scan_impl(const Tin* in, u64 n, u64* out, u64* d_total, char* ws, hipStream_t s) {
  if (n == 0) {
    if (d_total) set_u64_kernel<<<1, 1, 0, s>>>(d_total, 0);
    return hipGetLastError();
  }
  u64 nt = tiles_of(n);
  if (nt <= kSingleTiles) {
    // small: one block, tile after tile (fewer launches than reduce + scan)
    scan_down_kernel<Tin><<<1, kNT, 0, s>>>(in, n, nullptr, out, d_total, u32(nt));
    return hipGetLastError();
  }
  if (nt > 0x7fffffffULL) return hipErrorInvalidValue;
  u64* sums = reinterpret_cast<u64*>(ws);
  char* rest = ws + align_up(nt * sizeof(u64), 256);
  scan_reduce_kernel<Tin><<<dim3(u32(nt)), kNT, 0, s>>>(in, n, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // scan the tile sums in place (each element is read before it is written
  // by the same thread, and the reduce pass has finished before)
  u64* sums_scanned = reinterpret_cast<u64*>(rest);
  rest += align_up(nt * sizeof(u64), 256);
  e = scan_impl<u64>(sums, nt, sums_scanned, nullptr, rest, s);
  if (e != hipSuccess) return e;
  scan_down_kernel<Tin><<<dim3(u32(nt)), kNT, 0, s>>>(in, n, sums_scanned, out, d_total);
  return hipGetLastError();
}

}  // namespace

u64 scan_workspace_bytes(u64 n) {
  u64 total = 0;
  u64 m = n;
  while (tiles_of(m) > 1) {
    u64 nt = tiles_of(m);
    total += 2 * align_up(nt * sizeof(u64), 256);
    m = nt;
  }
  return total + 256;
}

hipError_t scan_u32_u64(const u32* in, u64 n, u64* out, u64* d_total, void* ws, hipStream_t s) {
  return scan_impl<u32>(in, n, out, d_total, static_cast<char*>(ws), s);
}

// u64 -> u64 scan, used internally by other launchers.
hipError_t scan_u64_u64(const u64* in, u64 n, u64* out, u64* d_total, void* ws, hipStream_t s) {
  return scan_impl<u64>(in, n, out, d_total, static_cast<char*>(ws), s);
}

}  // namespace hl
