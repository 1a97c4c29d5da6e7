// LSD radix sort of packed tuple keys (Section 3.2: the sorted index array
// orders tuples lexicographically with the join columns first; Algorithm 1
// stable-sorts one column at a time from the least significant one, which
// on a packed key is exactly an LSD radix sort over its bits).
//
// Only the significant low `bits` bits are sorted (2 x the id width for a
// pair), 8 bits per pass.  One pass: per-tile digit histogram, an
// exclusive scan of the digit-major count matrix, then a stable scatter in
// which each wave ranks its keys by 64-lane ballot matching, the tile is
// reordered by digit in LDS and written out in runs per digit.
#include "device.hpp"
#include "kernels.hpp"

namespace hl {

hipError_t scan_u64_u64(const u64* in, u64 n, u64* out, u64* d_total, void* ws, hipStream_t s);

namespace {

constexpr int kBits = 8;
constexpr int kBuckets = 1 << kBits;
constexpr int kNT = 256;
constexpr int kWaves = kNT / kWave;
constexpr int kItems = 16;
constexpr u64 kTile = u64(kNT) * kItems;
constexpr u32 kWaveTile = kWave * kItems;
static_assert(kNT == kBuckets, "one thread per digit bucket");

// Lanes of `valid` whose digit equals this lane's.
__device__ __forceinline__ u64 peers_of(u32 d, u64 valid) {
  u64 m = valid;
#pragma unroll
  for (int b = 0; b < kBits; ++b) {
    u64 bb = ballot((d >> b) & 1u);
    m &= ((d >> b) & 1u) ? bb : ~bb;
  }
  return m;
}

template <typename K>
__device__ __forceinline__ u32 digit(K k, int shift) {
  return u32(k >> shift) & (kBuckets - 1);
}

template <typename K>
__global__ __launch_bounds__(kNT) void rs_hist_kernel(const K* keys, u64 n, int shift, u32* counts,
                                                      u32 ntiles) {
  __shared__ u32 hist[kWaves * kBuckets];
  for (int i = threadIdx.x; i < kWaves * kBuckets; i += kNT) hist[i] = 0;
  __syncthreads();
  const u32 tile = xcd_tile(blockIdx.x, gridDim.x);
  const int w = threadIdx.x / kWave;
  const u64 base = u64(tile) * kTile + u64(w) * kWaveTile;
  u32* h = hist + w * kBuckets;
  const u64 lt = lanemask_lt();
  for (int j = 0; j < kItems; ++j) {
    u64 i = base + u64(j) * kWave + lane_id();
    bool valid = i < n;
    u32 d = valid ? digit(keys[i], shift) : 0u;
    u64 vm = ballot(valid);
    if (vm == 0) break;  // wave-uniform
    u64 peers = peers_of(d, vm);
    // one lane per distinct digit adds the group's size; groups of later
    // rounds read the value after this write (LDS is in order per wave)
    if (valid && (peers & lt) == 0) h[d] += u32(popc(peers));
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  const int d = threadIdx.x;
  u32 c = 0;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) c += hist[q * kBuckets + d];
  counts[u64(d) * ntiles + tile] = c;
}

template <typename K>
__global__ __launch_bounds__(kNT) void rs_scatter_kernel(const K* in, K* out, u64 n, int shift,
                                                         const u64* offsets, u32 ntiles) {
  __shared__ u32 whist[kWaves * kBuckets];
  __shared__ u32 dstart[kBuckets];
  __shared__ u64 gbase[kBuckets];
  __shared__ u32 wsum[kWaves];
  __shared__ K tile_keys[kTile];
  for (int i = threadIdx.x; i < kWaves * kBuckets; i += kNT) whist[i] = 0;
  __syncthreads();
  const u32 tile = xcd_tile(blockIdx.x, gridDim.x);
  const int w = threadIdx.x / kWave;
  const u64 tbase = u64(tile) * kTile;
  const u64 base = tbase + u64(w) * kWaveTile;
  u32* h = whist + w * kBuckets;
  const u64 lt = lanemask_lt();
  K key[kItems];
  u32 rank[kItems];
  // rank of each key among the equal-digit keys of this wave, in input order
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    u64 i = base + u64(j) * kWave + lane_id();
    bool valid = i < n;
    key[j] = valid ? in[i] : K(0);
    u32 d = digit(key[j], shift);
    u64 vm = ballot(valid);
    u64 peers = peers_of(d, vm);
    u32 pre = valid ? h[d] : 0u;
    rank[j] = pre + u32(popc(peers & lt));
    if (valid && (peers & lt) == 0) h[d] = pre + u32(popc(peers));
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  {
    const int d = threadIdx.x;
    u32 run = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
      u32 c = whist[q * kBuckets + d];
      whist[q * kBuckets + d] = run;  // keys of digit d in earlier waves
      run += c;
    }
    u32 tot;
    u32 ex = block_exclusive_scan<kNT>(run, wsum, tot);
    dstart[d] = ex;
    gbase[d] = offsets[u64(d) * ntiles + tile] - ex;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    u64 i = base + u64(j) * kWave + lane_id();
    if (i < n) {
      u32 d = digit(key[j], shift);
      tile_keys[dstart[d] + h[d] + rank[j]] = key[j];
    }
  }
  __syncthreads();
  const u64 cnt = (n - tbase) < kTile ? (n - tbase) : kTile;
  for (u32 p = threadIdx.x; p < cnt; p += kNT) {
    K k = tile_keys[p];
    out[gbase[digit(k, shift)] + p] = k;
  }
}

u64 tiles_of(u64 n) { return (n + kTile - 1) / kTile; }

}  // namespace

u64 sort_workspace_bytes(u64 n) {
  u64 nt = tiles_of(n);
  u64 m = u64(kBuckets) * nt;
  return align_up(m * sizeof(u32), 256) + align_up(m * sizeof(u64), 256) + scan_workspace_bytes(m);
}

template <typename K>
hipError_t radix_sort(K* keys, K* alt, u64 n, int bits, void* ws, hipStream_t s, K** sorted,
                      LaunchTimer* timer) {
  *sorted = keys;
  if (n <= 1 || bits <= 0) return hipSuccess;
  if (n >= (u64(1) << 32)) return hipErrorInvalidValue;
  if (bits > int(8 * sizeof(K))) bits = int(8 * sizeof(K));
  const u64 nt = tiles_of(n);
  const u64 m = u64(kBuckets) * nt;
  char* p = static_cast<char*>(ws);
  u32* counts = reinterpret_cast<u32*>(p);
  p += align_up(m * sizeof(u32), 256);
  u64* offsets = reinterpret_cast<u64*>(p);
  p += align_up(m * sizeof(u64), 256);
  K* src = keys;
  K* dst = alt;
  for (int shift = 0; shift < bits; shift += kBits) {
    if (timer) timer->begin(K_RADIX_HIST, s);
    rs_hist_kernel<K><<<dim3(u32(nt)), kNT, 0, s>>>(src, n, shift, counts, u32(nt));
    if (timer) timer->end(K_RADIX_HIST, s, n * sizeof(K) + m * sizeof(u32));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_u32_u64(counts, m, offsets, nullptr, p, s);
    if (e != hipSuccess) return e;
    if (timer) timer->begin(K_RADIX_SCATTER, s);
    rs_scatter_kernel<K><<<dim3(u32(nt)), kNT, 0, s>>>(src, dst, n, shift, offsets, u32(nt));
    if (timer) timer->end(K_RADIX_SCATTER, s, 2 * n * sizeof(K) + m * sizeof(u64));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    K* t = src;
    src = dst;
    dst = t;
  }
  *sorted = src;
  return hipSuccess;
}

template hipError_t radix_sort<u32>(u32*, u32*, u64, int, void*, hipStream_t, u32**,
                                    LaunchTimer*);
template hipError_t radix_sort<u64>(u64*, u64*, u64, int, void*, hipStream_t, u64**,
                                    LaunchTimer*);

}  // namespace hl
