// LSD radix sort of packed tuple keys (Section 4.2: the sorted index array
// orders tuples lexicographically with the join columns first; Algorithm 1
// stable-sorts one column at a time from the least significant one, which
// on a packed key is exactly an LSD radix sort over its bits).
//
// Only the significant low `bits` bits are sorted (2 x the id width for a
// pair), 8 bits per pass.  One pass:
//   1. per-tile digit histogram: LDS atomic adds into sub-histograms (one
//      per eighth of a wave, so a digit shared by a whole wave serialises 8
//      lanes, not 64), written tile-major so each tile writes one row;
//   2. column scan of the count matrix (chunk sums, a scan per digit over
//      the chunks, the digit bases, per-tile offsets), all coalesced;
//   3. stable scatter: each wave ranks its keys among the equal-digit keys
//      of the wave by matching digits with one ballot per digit bit, the
//      tile is reordered by digit in LDS and written out in runs per digit.
// The digit width of a pass is a compile-time constant, so the matching
// loop is straight-line code: per digit bit one sign-extending bit
// extract, one ballot and two three-input logic operations (v_bitop3) that
// narrow the 64-lane peer mask, and the rank is one masked bit count.
// Tiles whose keys all exist skip every bounds test.
// (A single-sweep variant with decoupled look-back was measured slower on
// this chip: the look-back walks over many in-flight tiles with
// fabric-latency loads.)
#include "device.hpp"
#include "kernels.hpp"

namespace hl {

namespace {

constexpr int kBits = 8;
constexpr int kBuckets = 1 << kBits;
constexpr int kNT = 256;
constexpr int kWaves = kNT / kWave;
constexpr u32 kChunk = 64;  // tiles per chunk of the column scan
static_assert(kNT == kBuckets, "one thread per digit bucket");

// Keys per thread of a tile (histogram and scatter use the same tiles):
// 32 (8,192-key tiles) by default, or 16 (4,096), a run-time choice that
// the autotuner measures.  Larger tiles spread the per-tile work of both
// kernels (count rows, sub-histogram clearing and reduction, the digit
// scan) over more keys, and each digit's run in a tile is longer, so the
// scatter's writes are less fragmented: on 2^28 32-bit keys 108 against 89
// Gkeys/s; on 5e8 64-bit keys 16.4 against 18.5 ms (the 64 KB LDS copy of a
// 64-bit tile leaves two workgroups per CU, which is enough).  Smaller
// sorts (2^24 keys and below) gain a little from the smaller tiles.
constexpr u64 kMinTile = u64(kNT) * 16;  // the smallest tile

// A pass sorts on bits [shift, shift + DB) of the key, DB <= 8.
template <int DB, typename K>
__device__ __forceinline__ u32 digit(K k, int shift) {
  return u32(k >> shift) & ((1u << DB) - 1u);
}

// Narrows the peer mask (lo, hi) to the lanes whose DB-bit digit equals
// this lane's: per bit b, t is 0 or ~0 by the lane's bit, B the ballot of
// that bit, and the lanes kept are those where B agrees with t:
// mask & ~(B ^ t), one v_bitop3 per half (truth table 0x90).
template <int DB>
__device__ __forceinline__ void match_digit(u32 d, u32& lo, u32& hi) {
#pragma unroll
  for (int b = 0; b < DB; ++b) {
    const u32 t = u32(__builtin_amdgcn_sbfe(int(d), b, 1));
    const u64 B = __builtin_amdgcn_uicmp(t, 0u, 33);  // ballot of t != 0
    lo = __builtin_amdgcn_bitop3_b32(lo, u32(B), t, 0x90);
    hi = __builtin_amdgcn_bitop3_b32(hi, u32(B >> 32), t, 0x90);
  }
}

// Lanes of the 64-bit mask (lo, hi) below this lane.
__device__ __forceinline__ u32 lanes_below(u32 lo, u32 hi) {
  return __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
}

// Per-tile digit histogram; counts are tile-major: counts[tile * 256 + d].
// No ranks are needed here, so keys are counted with LDS atomic adds rather
// than ballots.  Each eighth of a wave has its own sub-histogram (padded by
// one word so that equal digits of different eighths fall in different
// banks): a digit shared by every key of a wave serialises 8 lanes, not 64.
constexpr int kSubsPerWave = 8;
constexpr int kSubs = kWaves * kSubsPerWave;
constexpr int kSubStride = kBuckets + 1;
constexpr int kHistWords = (kSubs * kSubStride + 3) / 4 * 4;

template <typename K, int DB, int IT>
__global__ __launch_bounds__(kNT) void rs_hist_kernel(const K* keys, u64 n, int shift,
                                                      u32* counts, u32 ntiles) {
  constexpr u64 kTile = u64(kNT) * IT;
  constexpr u32 kWaveTile = kWave * IT;
  __shared__ __align__(16) u32 hist[kHistWords];
  {
    uint4* h4 = reinterpret_cast<uint4*>(hist);
    for (int i = threadIdx.x; i < kHistWords / 4; i += kNT) h4[i] = make_uint4(0, 0, 0, 0);
  }
  const u32 tile = xcd_tile(blockIdx.x, gridDim.x);
  const int w = threadIdx.x / kWave;
  const u64 base = u64(tile) * kTile + u64(w) * kWaveTile;
  const bool whole = u64(tile) * kTile + kTile <= n;
  // all loads first, so each wave has IT loads in flight
  K key[IT];
  if (whole) {
#pragma unroll
    for (int j = 0; j < IT; ++j) key[j] = keys[base + u64(j) * kWave + lane_id()];
  } else {
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const u64 i = base + u64(j) * kWave + lane_id();
      key[j] = i < n ? keys[i] : K(0);
    }
  }
  __syncthreads();
  u32* h = hist + (w * kSubsPerWave + lane_id() / (kWave / kSubsPerWave)) * kSubStride;
  if (whole) {
#pragma unroll
    for (int j = 0; j < IT; ++j) atomicAdd(&h[digit<DB>(key[j], shift)], 1u);
  } else {
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const u64 i = base + u64(j) * kWave + lane_id();
      if (i < n) atomicAdd(&h[digit<DB>(key[j], shift)], 1u);
    }
  }
  __syncthreads();
  const int d = threadIdx.x;
  u32 c = 0;
#pragma unroll
  for (int q = 0; q < kSubs; ++q) c += hist[q * kSubStride + d];
  counts[u64(tile) * kBuckets + d] = c;
}

// Column scan of the tile-major count matrix.
// 1. chunk sums: csum[c * 256 + d] = sum of counts[t * 256 + d] over the
//    tiles t of chunk c.
__global__ __launch_bounds__(kNT) void col_reduce_kernel(const u32* counts, u32 ntiles,
                                                         u32* csum) {
  const u32 c = blockIdx.x, d = threadIdx.x;
  const u32 t0 = c * kChunk, t1 = min(ntiles, t0 + kChunk);
  u32 s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  u32 t = t0;
  for (; t + 4 <= t1; t += 4) {
    s0 += counts[u64(t) * kBuckets + d];
    s1 += counts[u64(t + 1) * kBuckets + d];
    s2 += counts[u64(t + 2) * kBuckets + d];
    s3 += counts[u64(t + 3) * kBuckets + d];
  }
  for (; t < t1; ++t) s0 += counts[u64(t) * kBuckets + d];
  csum[u64(c) * kBuckets + d] = s0 + s1 + s2 + s3;
}

// 2. one block per digit: exclusive scan of that digit's column of chunk
//    sums (in place); the digit's total goes to total[d].
__global__ __launch_bounds__(kNT) void col_scan_kernel(u32* csum, u32 nchunks, u32* total) {
  __shared__ u32 wsum[kWaves];
  const u32 d = blockIdx.x;
  u32 carry = 0;
  for (u32 c0 = 0; c0 < nchunks; c0 += kNT) {
    const u32 c = c0 + threadIdx.x;
    const u32 v = c < nchunks ? csum[u64(c) * kBuckets + d] : 0u;
    u32 tot;
    const u32 ex = block_exclusive_scan<kNT>(v, wsum, tot);
    if (c < nchunks) csum[u64(c) * kBuckets + d] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) total[d] = carry;
}

// 3. digit bases (exclusive scan of the totals) and 4. per-tile offsets:
//    offsets[t * 256 + d] = base[d] + keys of digit d in earlier tiles.
__global__ __launch_bounds__(kNT) void col_offsets_kernel(const u32* counts, u32 ntiles,
                                                          const u32* csum, const u32* total,
                                                          u32* offsets) {
  __shared__ u32 wsum[kWaves];
  const u32 c = blockIdx.x, d = threadIdx.x;
  u32 tot;
  const u32 base = block_exclusive_scan<kNT>(total[d], wsum, tot);
  const u32 t0 = c * kChunk, t1 = min(ntiles, t0 + kChunk);
  u32 run = base + csum[u64(c) * kBuckets + d];
  for (u32 t = t0; t < t1; ++t) {
    const u32 v = counts[u64(t) * kBuckets + d];
    offsets[u64(t) * kBuckets + d] = run;
    run += v;
  }
}

// All of the above in one block, for at most one chunk of tiles (small
// sorts, where launches cost more than the work).
__global__ __launch_bounds__(kNT) void col_single_kernel(const u32* counts, u32 ntiles,
                                                         u32* offsets) {
  __shared__ u32 wsum[kWaves];
  const u32 d = threadIdx.x;
  u32 s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  u32 t = 0;
  for (; t + 4 <= ntiles; t += 4) {
    s0 += counts[u64(t) * kBuckets + d];
    s1 += counts[u64(t + 1) * kBuckets + d];
    s2 += counts[u64(t + 2) * kBuckets + d];
    s3 += counts[u64(t + 3) * kBuckets + d];
  }
  for (; t < ntiles; ++t) s0 += counts[u64(t) * kBuckets + d];
  u32 tot;
  u32 run = block_exclusive_scan<kNT>(s0 + s1 + s2 + s3, wsum, tot);
  for (t = 0; t < ntiles; ++t) {
    const u32 v = counts[u64(t) * kBuckets + d];
    offsets[u64(t) * kBuckets + d] = run;
    run += v;
  }
}

template <typename K, int DB, int IT>
__global__ __launch_bounds__(kNT) void rs_scatter_kernel(const K* in, K* out, u64 n, int shift,
                                                         const u32* offsets, u32 ntiles) {
  constexpr u64 kTile = u64(kNT) * IT;
  constexpr u32 kWaveTile = kWave * IT;
  __shared__ u32 whist[kWaves * kBuckets];
  __shared__ u32 gbase[kBuckets];
  __shared__ u32 wsum[kWaves];
  __shared__ K tile_keys[kTile];
  for (int i = threadIdx.x; i < kWaves * kBuckets; i += kNT) whist[i] = 0;
  const u32 tile = xcd_tile(blockIdx.x, gridDim.x);
  const int w = threadIdx.x / kWave;
  const u64 tbase = u64(tile) * kTile;
  const u64 base = tbase + u64(w) * kWaveTile;
  const bool whole = tbase + kTile <= n;
  K key[IT];
  if (whole) {
#pragma unroll
    for (int j = 0; j < IT; ++j) key[j] = in[base + u64(j) * kWave + lane_id()];
  } else {
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const u64 i = base + u64(j) * kWave + lane_id();
      key[j] = i < n ? in[i] : K(0);
    }
  }
  const u32 gofs = offsets[u64(tile) * kBuckets + threadIdx.x];
  __syncthreads();
  u32* h = whist + w * kBuckets;
  // rank of each key among the equal-digit keys of this wave, in input
  // order: the count of that digit in earlier rounds (h) plus the peers in
  // lower lanes; the lowest peer advances h
  u32 rank[IT];
  if (whole) {
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const u32 d = digit<DB>(key[j], shift);
      u32 lo = ~0u, hi = ~0u;
      match_digit<DB>(d, lo, hi);
      const u32 below = lanes_below(lo, hi);
      const u32 pre = h[d];
      rank[j] = pre + below;
      if (below == 0) h[d] = pre + u32(__popc(lo)) + u32(__popc(hi));
      __builtin_amdgcn_wave_barrier();
    }
  } else {
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const bool valid = base + u64(j) * kWave + lane_id() < n;
      const u64 vm = ballot(valid);
      const u32 d = digit<DB>(key[j], shift);
      u32 lo = u32(vm), hi = u32(vm >> 32);
      match_digit<DB>(d, lo, hi);
      const u32 below = lanes_below(lo, hi);
      const u32 pre = h[d];
      rank[j] = pre + below;
      if (valid && below == 0) h[d] = pre + u32(__popc(lo)) + u32(__popc(hi));
      __builtin_amdgcn_wave_barrier();
    }
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
    // each wave's slot of digit d: the digit's start in the tile plus the
    // keys of digit d in earlier waves (one LDS read per key below)
#pragma unroll
    for (int q = 0; q < kWaves; ++q) whist[q * kBuckets + d] += ex;
    gbase[d] = gofs - ex;  // modular: gbase + p is the global position
  }
  __syncthreads();
  if (whole) {
#pragma unroll
    for (int j = 0; j < IT; ++j) tile_keys[h[digit<DB>(key[j], shift)] + rank[j]] = key[j];
  } else {
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const u64 i = base + u64(j) * kWave + lane_id();
      if (i < n) tile_keys[h[digit<DB>(key[j], shift)] + rank[j]] = key[j];
    }
  }
  __syncthreads();
  if (whole) {
    // kTile = IT * kNT positions
#pragma unroll 8
    for (int j = 0; j < IT; ++j) {
      const u32 p = u32(j) * kNT + threadIdx.x;
      const K k = tile_keys[p];
      out[u32(gbase[digit<DB>(k, shift)] + p)] = k;
    }
  } else {
    const u32 cnt = u32(n - tbase);
    for (u32 p = threadIdx.x; p < cnt; p += kNT) {
      const K k = tile_keys[p];
      out[u32(gbase[digit<DB>(k, shift)] + p)] = k;
    }
  }
}

u64 tiles_of(u64 n, int items) {
  const u64 t = u64(kNT) * u64(items);
  return (n + t - 1) / t;
}

// One pass over bits [shift, shift + DB) with tiles of IT keys per thread.
template <typename K, int DB, int IT>
hipError_t rs_pass(const K* src, K* dst, u64 n, int shift, u32* counts, u32* offsets, u32* csum,
                   u32* total, u64 nt, u64 nc, hipStream_t s, LaunchTimer* timer) {
  const u64 m = u64(kBuckets) * nt;
  if (timer) timer->begin(K_RADIX_HIST, s);
  rs_hist_kernel<K, DB, IT><<<dim3(u32(nt)), kNT, 0, s>>>(src, n, shift, counts, u32(nt));
  if (timer) timer->end(K_RADIX_HIST, s, n * sizeof(K) + m * sizeof(u32));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nc == 1) {
    col_single_kernel<<<1, kNT, 0, s>>>(counts, u32(nt), offsets);
  } else {
    col_reduce_kernel<<<dim3(u32(nc)), kNT, 0, s>>>(counts, u32(nt), csum);
    col_scan_kernel<<<dim3(kBuckets), kNT, 0, s>>>(csum, u32(nc), total);
    col_offsets_kernel<<<dim3(u32(nc)), kNT, 0, s>>>(counts, u32(nt), csum, total, offsets);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (timer) timer->begin(K_RADIX_SCATTER, s);
  rs_scatter_kernel<K, DB, IT><<<dim3(u32(nt)), kNT, 0, s>>>(src, dst, n, shift, offsets,
                                                             u32(nt));
  if (timer) timer->end(K_RADIX_SCATTER, s, 2 * n * sizeof(K) + m * sizeof(u32));
  return hipGetLastError();
}

}  // namespace

u64 sort_workspace_bytes(u64 n) {
  // sized for the smallest tile (the most count rows) of any key type
  const u64 nt = (n + kMinTile - 1) / kMinTile;
  const u64 nc = (nt + kChunk - 1) / kChunk;
  return 2 * align_up(nt * kBuckets * sizeof(u32), 256) +
         align_up(nc * kBuckets * sizeof(u32), 256) + align_up(kBuckets * sizeof(u32), 256);
}

template <typename K>
hipError_t radix_sort_bits(K* keys, K* alt, u64 n, int lo_bit, int hi_bit, void* ws,
                           hipStream_t s, K** sorted, LaunchTimer* timer, int tile_items) {
  *sorted = keys;
  if (hi_bit > int(8 * sizeof(K))) hi_bit = int(8 * sizeof(K));
  if (n <= 1 || lo_bit < 0 || hi_bit <= lo_bit) return hipSuccess;
  if (n >= (u64(1) << 32)) return hipErrorInvalidValue;
  if (tile_items != 16 && tile_items != 32) return hipErrorInvalidValue;
  const u64 nt = tiles_of(n, tile_items);
  const u64 nc = (nt + kChunk - 1) / kChunk;
  const u64 m = u64(kBuckets) * nt;
  char* p = static_cast<char*>(ws);
  u32* counts = reinterpret_cast<u32*>(p);
  p += align_up(m * sizeof(u32), 256);
  u32* offsets = reinterpret_cast<u32*>(p);
  p += align_up(m * sizeof(u32), 256);
  u32* csum = reinterpret_cast<u32*>(p);
  p += align_up(nc * kBuckets * sizeof(u32), 256);
  u32* total = reinterpret_cast<u32*>(p);
  K* src = keys;
  K* dst = alt;
  for (int shift = lo_bit; shift < hi_bit; shift += kBits) {
    const int dbits = (hi_bit - shift) < kBits ? (hi_bit - shift) : kBits;
    hipError_t e = hipSuccess;
#define HL_RS_PASS(DB)                                                                        \
  case DB:                                                                                    \
    e = tile_items == 32                                                                      \
            ? rs_pass<K, DB, 32>(src, dst, n, shift, counts, offsets, csum, total, nt, nc, s, \
                                 timer)                                                       \
            : rs_pass<K, DB, 16>(src, dst, n, shift, counts, offsets, csum, total, nt, nc, s, \
                                 timer);                                                      \
    break;
    switch (dbits) {
      HL_RS_PASS(1)
      HL_RS_PASS(2)
      HL_RS_PASS(3)
      HL_RS_PASS(4)
      HL_RS_PASS(5)
      HL_RS_PASS(6)
      HL_RS_PASS(7)
      HL_RS_PASS(8)
      default:
        return hipErrorInvalidValue;
    }
#undef HL_RS_PASS
    if (e != hipSuccess) return e;
    K* t = src;
    src = dst;
    dst = t;
  }
  *sorted = src;
  return hipSuccess;
}

template <typename K>
hipError_t radix_sort(K* keys, K* alt, u64 n, int bits, void* ws, hipStream_t s, K** sorted,
                      LaunchTimer* timer, int tile_items) {
  return radix_sort_bits<K>(keys, alt, n, 0, bits, ws, s, sorted, timer, tile_items);
}

template hipError_t radix_sort<u32>(u32*, u32*, u64, int, void*, hipStream_t, u32**,
                                    LaunchTimer*, int);
template hipError_t radix_sort<u64>(u64*, u64*, u64, int, void*, hipStream_t, u64**,
                                    LaunchTimer*, int);
template hipError_t radix_sort_bits<u32>(u32*, u32*, u64, int, int, void*, hipStream_t, u32**,
                                         LaunchTimer*, int);
template hipError_t radix_sort_bits<u64>(u64*, u64*, u64, int, int, void*, hipStream_t, u64**,
                                         LaunchTimer*, int);

}  // namespace hl
