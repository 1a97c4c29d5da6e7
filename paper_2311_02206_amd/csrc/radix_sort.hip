// LSD radix sort of packed tuple keys (Section 3.2: the sorted index array
// orders tuples lexicographically with the join columns first; Algorithm 1
// stable-sorts one column at a time from the least significant one, which
// on a packed key is exactly an LSD radix sort over its bits).
//
// Only the significant low `bits` bits are sorted (2 x the id width for a
// pair), 8 bits per pass, in the single-sweep form of Adinets and Merrill
// ("Onesweep", 2022):
//   1. one read of the keys builds the global digit histogram of every pass;
//   2. one kernel per pass: each workgroup claims the next tile in order
//      from an atomic counter, ranks its keys by 64-lane ballot matching,
//      publishes its per-digit counts, adds up the counts (or the inclusive
//      prefixes) of the tiles before it by decoupled look-back, and writes
//      its keys, reordered by digit in LDS, to their final positions.
// Each pass reads and writes every key once.  A waiting tile only waits on
// tiles that were claimed before it (so are running) and that publish
// their counts before they wait themselves; every wait is also bounded, and
// a wait that runs out sets an error flag instead of hanging.
#include "device.hpp"
#include "kernels.hpp"

namespace hl {

namespace {

constexpr int kBits = 8;
constexpr int kBuckets = 1 << kBits;
constexpr int kNT = 256;
constexpr int kWaves = kNT / kWave;
constexpr int kItems = 16;
constexpr u64 kTile = u64(kNT) * kItems;
constexpr u32 kWaveTile = kWave * kItems;
constexpr int kMaxPasses = 8;
static_assert(kNT == kBuckets, "one thread per digit bucket");

// Look-back status word: [63:62] state (0 none, 1 tile count, 2 inclusive
// prefix), [61:56] pass tag, [55:0] value.
constexpr u64 kStAgg = u64(1) << 62;
constexpr u64 kStInc = u64(2) << 62;
constexpr u64 kValMask = (u64(1) << 56) - 1;
constexpr u32 kSpinLimit = 1u << 22;

__device__ __forceinline__ u64 st_word(u64 state, u32 tag, u64 v) {
  return state | (u64(tag) << 56) | v;
}

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

// Global histogram of every pass (per-wave LDS sub-histograms).
template <typename K>
__global__ __launch_bounds__(kNT) void os_hist_kernel(const K* keys, u64 n, int npass,
                                                      u32* ghist) {
  __shared__ u32 h[kWaves * kMaxPasses * kBuckets];
  for (int i = threadIdx.x; i < kWaves * kMaxPasses * kBuckets; i += kNT) h[i] = 0;
  __syncthreads();
  u32* hw = h + (threadIdx.x / kWave) * kMaxPasses * kBuckets;
  const u64 stride = u64(gridDim.x) * kNT;
  for (u64 i = u64(blockIdx.x) * kNT + threadIdx.x; i < n; i += stride) {
    const K k = keys[i];
    for (int p = 0; p < npass; ++p) atomicAdd(&hw[p * kBuckets + digit(k, p * kBits)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < npass * kBuckets; i += kNT) {
    u32 c = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) c += h[q * kMaxPasses * kBuckets + i];
    if (c) atomicAdd(&ghist[i], c);
  }
}

// Exclusive scan over the digits of every pass: base[p][d].
__global__ __launch_bounds__(kNT) void os_base_kernel(const u32* ghist, int npass, u32* base) {
  __shared__ u32 wsum[kWaves];
  for (int p = 0; p < npass; ++p) {
    u32 tot;
    u32 ex = block_exclusive_scan<kNT>(ghist[p * kBuckets + threadIdx.x], wsum, tot);
    base[p * kBuckets + threadIdx.x] = ex;
  }
}

template <typename K>
__global__ __launch_bounds__(kNT) void os_scatter_kernel(const K* in, K* out, u64 n, int shift,
                                                         const u32* base, u64* status, u32 tag,
                                                         u32* tile_counter, u32* err) {
  __shared__ u32 whist[kWaves * kBuckets];
  __shared__ u32 dstart[kBuckets];
  __shared__ u32 gbase[kBuckets];
  __shared__ u32 wsum[kWaves];
  __shared__ u32 s_tile;
  __shared__ K tile_keys[kTile];
  for (int i = threadIdx.x; i < kWaves * kBuckets; i += kNT) whist[i] = 0;
  if (threadIdx.x == 0) s_tile = atomicAdd(tile_counter, 1u);
  __syncthreads();
  const u32 tile = s_tile;
  const int w = threadIdx.x / kWave;
  const u64 tbase = u64(tile) * kTile;
  const u64 wbase = tbase + u64(w) * kWaveTile;
  K key[kItems];
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    u64 i = wbase + u64(j) * kWave + lane_id();
    key[j] = i < n ? in[i] : K(0);
  }
  u32* h = whist + w * kBuckets;
  const u64 lt = lanemask_lt();
  u32 rank[kItems];
  // rank of each key among the equal-digit keys of this wave, in input order
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    u64 i = wbase + u64(j) * kWave + lane_id();
    bool valid = i < n;
    u32 d = digit(key[j], shift);
    u64 vm = ballot(valid);
    u64 peers = peers_of(d, vm);
    u32 pre = valid ? h[d] : 0u;
    rank[j] = pre + u32(popc(peers & lt));
    if (valid && (peers & lt) == 0) h[d] = pre + u32(popc(peers));
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  const int d = threadIdx.x;
  u32 cnt_d = 0;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) {
    u32 c = whist[q * kBuckets + d];
    whist[q * kBuckets + d] = cnt_d;  // keys of digit d in earlier waves
    cnt_d += c;
  }
  // publish this tile's count of digit d, then look back for the prefix
  u64* row = status + u64(tile) * kBuckets;
  u64 excl = 0;
  if (tile == 0) {
    __hip_atomic_store(&row[d], st_word(kStInc, tag, cnt_d), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  } else {
    __hip_atomic_store(&row[d], st_word(kStAgg, tag, cnt_d), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    u32 spins = 0;
    for (u64 t = tile - 1;; --t) {
      u64 v = __hip_atomic_load(&status[t * kBuckets + d], __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
      while ((v >> 62) == 0 || u32((v >> 56) & 63) != tag) {
        if (++spins > kSpinLimit) {
          atomicOr(err, 1u);
          v = st_word(kStInc, tag, 0);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        v = __hip_atomic_load(&status[t * kBuckets + d], __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
      }
      excl += v & kValMask;
      if ((v >> 62) == 2 || t == 0) break;
    }
    __hip_atomic_store(&row[d], st_word(kStInc, tag, excl + cnt_d), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  {
    u32 tot;
    u32 ex = block_exclusive_scan<kNT>(cnt_d, wsum, tot);
    dstart[d] = ex;
    gbase[d] = base[d] + u32(excl) - ex;  // modular: gbase + p is the position
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    u64 i = wbase + u64(j) * kWave + lane_id();
    if (i < n) {
      u32 dd = digit(key[j], shift);
      tile_keys[dstart[dd] + h[dd] + rank[j]] = key[j];
    }
  }
  __syncthreads();
  const u32 cnt = u32((n - tbase) < kTile ? (n - tbase) : kTile);
  for (u32 p = threadIdx.x; p < cnt; p += kNT) {
    K k = tile_keys[p];
    out[u32(gbase[digit(k, shift)] + p)] = k;
  }
}

__global__ void or_err_kernel(const u32* err, u32* dst) {
  if (*err) *dst |= *err;
}

u64 tiles_of(u64 n) { return (n + kTile - 1) / kTile; }

// Workspace layout: status rows, then the small arrays.
struct Layout {
  u64 status, ghist, base, counters, err, total;
};

Layout layout_of(u64 n) {
  Layout L;
  u64 off = 0;
  L.status = off;
  off += align_up(tiles_of(n) * kBuckets * sizeof(u64), 256);
  L.ghist = off;
  off += align_up(kMaxPasses * kBuckets * sizeof(u32), 256);
  L.base = off;
  off += align_up(kMaxPasses * kBuckets * sizeof(u32), 256);
  L.counters = off;
  off += 256;
  L.err = off;
  off += 256;
  L.total = off;
  return L;
}

}  // namespace

u64 sort_workspace_bytes(u64 n) { return layout_of(n).total; }

template <typename K>
hipError_t radix_sort(K* keys, K* alt, u64 n, int bits, void* ws, hipStream_t s, K** sorted,
                      LaunchTimer* timer, u32* d_err) {
  *sorted = keys;
  if (n <= 1 || bits <= 0) return hipSuccess;
  if (n >= (u64(1) << 32)) return hipErrorInvalidValue;
  if (bits > int(8 * sizeof(K))) bits = int(8 * sizeof(K));
  const int npass = (bits + kBits - 1) / kBits;
  const u64 nt = tiles_of(n);
  const Layout L = layout_of(n);
  char* p = static_cast<char*>(ws);
  u64* status = reinterpret_cast<u64*>(p + L.status);
  u32* ghist = reinterpret_cast<u32*>(p + L.ghist);
  u32* base = reinterpret_cast<u32*>(p + L.base);
  u32* counters = reinterpret_cast<u32*>(p + L.counters);
  u32* err = reinterpret_cast<u32*>(p + L.err);
  hipError_t e = fill_zero(p, L.total, s);
  if (e != hipSuccess) return e;
  u64 hist_blocks = nt < 2048 ? nt : 2048;
  if (timer) timer->begin(K_RADIX_HIST, s);
  os_hist_kernel<K><<<dim3(u32(hist_blocks)), kNT, 0, s>>>(keys, n, npass, ghist);
  if (timer) timer->end(K_RADIX_HIST, s, n * sizeof(K));
  os_base_kernel<<<1, kNT, 0, s>>>(ghist, npass, base);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  K* src = keys;
  K* dst = alt;
  for (int pass = 0; pass < npass; ++pass) {
    if (timer) timer->begin(K_RADIX_SCATTER, s);
    os_scatter_kernel<K><<<dim3(u32(nt)), kNT, 0, s>>>(src, dst, n, pass * kBits,
                                                       base + pass * kBuckets, status,
                                                       u32(pass + 1), counters + pass, err);
    if (timer) timer->end(K_RADIX_SCATTER, s, 2 * n * sizeof(K));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    K* t = src;
    src = dst;
    dst = t;
  }
  if (d_err) {
    or_err_kernel<<<1, 1, 0, s>>>(err, d_err);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  *sorted = src;
  return hipSuccess;
}

template hipError_t radix_sort<u32>(u32*, u32*, u64, int, void*, hipStream_t, u32**,
                                    LaunchTimer*, u32*);
template hipError_t radix_sort<u64>(u64*, u64*, u64, int, void*, hipStream_t, u64**,
                                    LaunchTimer*, u32*);

}  // namespace hl
