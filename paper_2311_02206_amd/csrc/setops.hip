// Set operations on sorted key arrays.
//
// unique_diff: populating delta (Section 5.1, "Populating delta"): the
// sorted new tuples are deduplicated by comparing each with its neighbour
// (Section 4.2, "Deduplication") and every tuple already in full is
// removed, so delta and full stay disjoint.  Membership in full is a binary
// search restricted to the slice of full spanned by the tile, staged in
// LDS when it is small, else run for all of a thread's keys in lockstep.
//
// merge: full := full U delta by merge path (Section 4.2, "Merge
// operation", after Green, McColl and Bader 2012): a diagonal search splits
// the output into equal tiles, each tile merges its two input slices in
// LDS and writes its output with coalesced stores.
#include "device.hpp"
#include "kernels.hpp"

namespace hl {

hipError_t scan_u64_u64(const u64* in, u64 n, u64* out, u64* d_total, void* ws, hipStream_t s);

namespace {

// ------------------------------------------------------------ unique_diff

constexpr int kUdNT = 256;
// Candidates per thread of a tile: 16 (4,096-candidate tiles) by default, or
// 8 (2,048), a run-time choice that the autotuner measures.
constexpr u64 kUdMinTile = u64(kUdNT) * 8;
constexpr u64 kUdStage = 2048;  // keys of full staged in LDS per chunk
constexpr int kUdLock = 8;      // keys searched in lockstep by one thread
constexpr u64 kUdStreamMax = 16 * kUdStage;  // longest slice streamed through LDS

// One padding slot per ITEMS keys: thread t reads keys t*ITEMS .. t*ITEMS +
// ITEMS - 1, which without padding would all fall in the same LDS banks.
template <int ITEMS>
__device__ __forceinline__ u32 pad(u32 i) {
  return i + i / ITEMS;
}

template <typename K>
__device__ __forceinline__ u64 lower_bound(const K* a, u64 lo, u64 hi, K x) {
  while (lo < hi) {
    u64 mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <typename K>
__device__ __forceinline__ u64 upper_bound(const K* a, u64 lo, u64 hi, K x) {
  while (lo < hi) {
    u64 mid = (lo + hi) >> 1;
    if (!(x < a[mid])) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// part[2t] = lower_bound(full, first candidate of tile t) and part[2t + 1] =
// lower_bound(full, last candidate of tile t): every candidate of the tile
// has its lower bound between them, so the tile searches only that slice
// (keys of full between two tiles' candidates are never read).  One thread
// per bound, so the searches' latency overlaps across tiles.
template <typename K, bool kModel>
__global__ __launch_bounds__(kUdNT) void ud_partition_kernel(const K* cand, u64 n, const K* full,
                                                             u64 nf, u64 ntiles, u64 tile_keys,
                                                             u64* part, LearnedView<K> lv) {
  const u64 u = u64(blockIdx.x) * kUdNT + threadIdx.x;
  if (u >= 2 * ntiles) return;
  const u64 t = u >> 1;
  const u64 end = (t + 1) * tile_keys < n ? (t + 1) * tile_keys : n;
  const K x = (u & 1) ? cand[end - 1] : cand[t * tile_keys];
  part[u] = kModel ? u64(lm_lower_bound(lv, x)) : lower_bound(full, u64(0), nf, x);
}

// One tile of sorted candidates: each thread takes kUdItems consecutive
// keys, marks the first of each run of equal keys, and tests membership in
// the slice of full the tile spans.  A slice of up to kUdStreamMax keys is
// streamed through LDS in chunks of kUdStage keys, and each key is resolved
// in the first chunk whose last key is not below it (the keys of earlier
// chunks are all smaller); a longer slice is searched in global memory by
// lockstep searches.  One block scan places the survivors, which are written
// compacted (in order) at the tile's start in tmp.  The tile's kept and
// distinct counts go to tile_counts and tile_uniq.
// With alg_bytes (kernel timing), the tile adds the bytes its step must move
// by definition: its candidates read, its survivors written, and for the
// membership tests the cheaper of reading the slice of full it spans and
// one 64-byte line per distinct key searched (the same for the tail).
template <typename K, bool kModel, int kUdItems>
__global__ __launch_bounds__(kUdNT)
__attribute__((amdgpu_waves_per_eu(sizeof(K) == 4 && !kModel ? 6 : 1)))
void ud_select_kernel(const K* cand, u64 n, const K* full, u64 nf, K* tmp, u32* tile_counts,
                      u32* tile_uniq, LearnedView<K> lv, const u64* part, const K* tail,
                      u64 ntail, u64* alg_bytes,
                      u64* lockstep_tiles) {
  constexpr u64 kUdTile = u64(kUdNT) * kUdItems;
  __shared__ u32 wsum[kUdNT / kWave];
  __shared__ K s_c[kUdTile + kUdTile / kUdItems];
  __shared__ K staged[kUdStage];
  const u32 tile = blockIdx.x;
  const u64 base = u64(tile) * kUdTile;
  const u32 cnt = u32((n - base) < kUdTile ? (n - base) : kUdTile);
  // every candidate of the tile lies between the tile's first and last
  // keys, so its lower bound in full is in this slice (one past the last
  // key's lower bound, so that key's equal in full is in it too).  Each
  // thread reads the bounds itself (one address for the whole block), so
  // the first chunk of the slice can be requested together with the
  // candidates instead of after a barrier.
  const u64 lo = part[2 * u64(tile)];
  const u64 hi = (part[2 * u64(tile) + 1] + 1) < nf ? (part[2 * u64(tile) + 1] + 1) : nf;
  const K before = base > 0 ? cand[base - 1] : K(0);
  const u64 m = hi - lo;
  if (m > kUdStreamMax && lockstep_tiles && threadIdx.x == 0)
    atomicAdd(reinterpret_cast<unsigned long long*>(lockstep_tiles), 1ull);
  // the tile's candidates: every load issued before any is used (a loop
  // that stores each into LDS as it arrives waits out one memory latency
  // per key)
  K cv[kUdItems];
#pragma unroll
  for (int q = 0; q < kUdItems; ++q) {
    const u32 k = u32(q) * kUdNT + threadIdx.x;
    cv[q] = k < cnt ? cand[base + k] : K(0);
  }
  constexpr int kPer = int(kUdStage / kUdNT);
  K next[kPer];
  if (m <= kUdStreamMax) {
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const u64 i = lo + u64(r) * kUdNT + threadIdx.x;
      next[r] = i < hi ? full[i] : K(0);
    }
  }
#pragma unroll
  for (int q = 0; q < kUdItems; ++q) {
    const u32 k = u32(q) * kUdNT + threadIdx.x;
    if (k < cnt) s_c[pad<kUdItems>(k)] = cv[q];
  }
  // the slice's first chunk goes to LDS under the same barrier as the
  // candidates (most slices are one chunk: no barrier of their own)
  if (m <= kUdStreamMax) {
#pragma unroll
    for (int r = 0; r < kPer; ++r) staged[r * kUdNT + threadIdx.x] = next[r];
  }
  __syncthreads();
  const u32 b = threadIdx.x * kUdItems;
  u32 keep_bits = 0, nkeep = 0, uniq = 0;
  if (m <= kUdStreamMax) {
    // first-of-run flags, then resolution chunk by chunk
    u32 first_bits = 0;
    if (b < cnt) {
      K prevk = b > 0 ? s_c[pad<kUdItems>(b - 1)] : before;
#pragma unroll
      for (int q = 0; q < kUdItems; ++q) {
        const u32 idx = b + q;
        if (idx < cnt) {
          const K c = s_c[pad<kUdItems>(idx)];
          if ((base + idx == 0) || prevk != c) first_bits |= 1u << q;
          prevk = c;
        }
      }
    }
    uniq = u32(__popc(first_bits));
    u32 pending = first_bits;  // distinct keys not yet resolved
    // each thread holds its share of the next chunk in registers, loaded
    // while the current chunk is searched (the first one is already in LDS)
    for (u64 c0 = lo; c0 < hi; c0 += kUdStage) {  // block-uniform trip count
      const u32 cm = u32((hi - c0) < kUdStage ? (hi - c0) : kUdStage);
      if (c0 != lo) {
        __syncthreads();  // the previous chunk is no longer read
#pragma unroll
        for (int r = 0; r < kPer; ++r) staged[r * kUdNT + threadIdx.x] = next[r];
        __syncthreads();
      }
      const u64 c1 = c0 + kUdStage;
      if (c1 < hi) {
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
          const u64 i = c1 + u64(r) * kUdNT + threadIdx.x;
          next[r] = i < hi ? full[i] : K(0);
        }
      }
      if (pending) {
        const K clast = staged[cm - 1];
        const int q0 = __ffs(pending) - 1;
        if (s_c[pad<kUdItems>(b + q0)] <= clast) {
          // search the first pending key, walk forward for the others
          u32 p = u32(lower_bound(staged, u64(0), u64(cm), s_c[pad<kUdItems>(b + q0)]));
          for (int q = q0; q < kUdItems; ++q) {
            if (!(pending & (1u << q))) continue;
            const K c = s_c[pad<kUdItems>(b + q)];
            if (c > clast) break;
            while (staged[p] < c) ++p;  // stops at or before cm - 1
            pending &= ~(1u << q);
            if (staged[p] != c) {
              keep_bits |= 1u << q;
              ++nkeep;
            }
          }
        }
      }
    }
    // keys above the whole slice are not in full
    keep_bits |= pending;
    nkeep += u32(__popc(pending));
  } else if (b < cnt) {
    // The slice is too long to stream, so candidates may be far apart in
    // full.  Only the distinct keys of a thread are searched, in groups of
    // kUdLock whose halving steps run together, so a wave keeps many loads
    // in flight instead of forming one chain of dependent reads.  Every key
    // of a group has a search range of the same length L (the tile's slice,
    // or the widest of the model's windows intersected with it), so the
    // steps are the same for all.
    K prevk = b > 0 ? s_c[pad<kUdItems>(b - 1)] : before;
    int qd[kUdItems];
    int nd = 0;
#pragma unroll
    for (int q = 0; q < kUdItems; ++q) {
      const u32 idx = b + q;
      if (idx < cnt) {
        const K c = s_c[pad<kUdItems>(idx)];
        if ((base + idx == 0) || prevk != c) qd[nd++] = q;
        prevk = c;
      }
    }
    uniq = u32(nd);
#pragma unroll 1
    for (int g = 0; g < nd; g += kUdLock) {
      K c[kUdLock];
      const K* at[kUdLock];
      u64 L = m;
#pragma unroll
      for (int r = 0; r < kUdLock; ++r) {
        c[r] = s_c[pad<kUdItems>(b + qd[(g + r < nd) ? g + r : nd - 1])];
        at[r] = full + lo;
      }
      if (kModel) {
        // the model's window and the tile's slice both hold each key's
        // lower bound, so their intersection does too
        u64 wa[kUdLock];
        L = 0;
#pragma unroll
        for (int r = 0; r < kUdLock; ++r) {
          u64 wb;
          lm_window(lv, c[r], wa[r], wb);
          wa[r] = wa[r] > lo ? wa[r] : lo;
          wb = wb < hi ? wb : hi;
          if (wb < wa[r]) wb = wa[r];
          L = (wb - wa[r]) > L ? (wb - wa[r]) : L;
        }
        // widening a window keeps the answer inside it; stay within full
#pragma unroll
        for (int r = 0; r < kUdLock; ++r) at[r] = full + (wa[r] < nf - L ? wa[r] : nf - L);
      }
      u64 len = L;
      while (len > 1) {
        const u64 half = len >> 1;
#pragma unroll
        for (int r = 0; r < kUdLock; ++r) at[r] = (at[r][half] < c[r]) ? at[r] + half : at[r];
        len -= half;
      }
#pragma unroll
      for (int r = 0; r < kUdLock; ++r) {
        if (g + r < nd) {
          const u64 pos = u64(at[r] - full) + ((L > 0 && *at[r] < c[r]) ? 1 : 0);
          if (!(pos < nf && full[pos] == c[r])) {
            keep_bits |= 1u << qd[g + r];
            ++nkeep;
          }
        }
      }
    }
  }
  // A short sorted tail run kept beside full (disjoint from it): the keys
  // that survived full are searched there too, kUdLock at a time in
  // lockstep.
  const u32 tail_searched = ntail > 0 ? nkeep : 0u;
  if (ntail > 0) {
    u32 rem = keep_bits;
    while (rem) {
      K c[kUdLock];
      int qi[kUdLock];
      int k = 0;
#pragma unroll
      for (int j = 0; j < kUdLock; ++j) {
        if (rem) {
          const int q = __ffs(rem) - 1;
          rem &= rem - 1;
          qi[j] = q;
          c[j] = s_c[pad<kUdItems>(b + q)];
          k = j + 1;
        } else {
          qi[j] = -1;
          c[j] = K(0);
        }
      }
      const K* at[kUdLock];
#pragma unroll
      for (int j = 0; j < kUdLock; ++j) at[j] = tail;
      u64 len = ntail;
      while (len > 1) {
        const u64 half = len >> 1;
#pragma unroll
        for (int j = 0; j < kUdLock; ++j)
          if (j < k) at[j] = (at[j][half] < c[j]) ? at[j] + half : at[j];
        len -= half;
      }
#pragma unroll
      for (int j = 0; j < kUdLock; ++j) {
        if (j < k) {
          const u64 p = u64(at[j] - tail) + ((*at[j] < c[j]) ? 1 : 0);
          if (p < ntail && tail[p] == c[j]) {
            keep_bits &= ~(1u << qi[j]);
            --nkeep;
          }
        }
      }
    }
  }
  // One block scan serves two counts: kept keys (their exclusive prefix
  // places the survivors) and distinct keys, each at most one tile (below
  // 2^16), in the two halves of a word.
  static_assert(kUdTile < (u64(1) << 16), "tile counts share one word");
  u32 packed_total;
  const u32 packed = block_exclusive_scan<kUdNT>(nkeep | (uniq << 16), wsum, packed_total);
  u32 pos = packed & 0xffffu;
  const u32 total = packed_total & 0xffffu;
  uniq = packed_total >> 16;
  // survivors go back into s_c at their compacted positions (all reads of
  // s_c happened before the scan's barriers), then out coalesced
  K mine[kUdItems];
#pragma unroll
  for (int q = 0; q < kUdItems; ++q) mine[q] = (b + q < cnt) ? s_c[pad<kUdItems>(b + q)] : K(0);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kUdItems; ++q)
    if (keep_bits & (1u << q)) s_c[pad<kUdItems>(pos++)] = mine[q];
  __syncthreads();
  for (u32 k = threadIdx.x; k < total; k += kUdNT) tmp[base + k] = s_c[pad<kUdItems>(k)];
  u32 searched = 0;
  if (alg_bytes) searched = block_sum<kUdNT>(tail_searched, wsum);
  if (threadIdx.x == 0) {
    tile_counts[tile] = total;
    tile_uniq[tile] = uniq;
    if (alg_bytes) {
      const u64 full_b = m * sizeof(K) < u64(uniq) * 64 ? m * sizeof(K) : u64(uniq) * 64;
      const u64 tail_b =
          ntail * sizeof(K) < u64(searched) * 64 ? ntail * sizeof(K) : u64(searched) * 64;
      atomicAdd(reinterpret_cast<unsigned long long*>(alg_bytes),
                static_cast<unsigned long long>(u64(cnt + total) * sizeof(K) + full_b + tail_b));
    }
  }
}

template <typename K>
__global__ __launch_bounds__(kUdNT) void ud_gather_kernel(const K* tmp, const u32* tile_counts,
                                                          const u64* tile_off, u64 tile_keys,
                                                          const u64* tile_src, K* out) {
  const u32 tile = blockIdx.x;
  const u32 c = tile_counts[tile];
  // a tile's survivors start at its first candidate's index (tile_src), or
  // at the tile's own start when tiles hold a fixed number of candidates
  const u64 src = tile_src ? tile_src[tile] : u64(tile) * tile_keys;
  const u64 dst = tile_off[tile];
  // at most 16 keys per thread (the largest tile), loaded before any store
  K v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const u32 k = u32(q) * kUdNT + threadIdx.x;
    v[q] = k < c ? tmp[src + k] : K(0);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const u32 k = u32(q) * kUdNT + threadIdx.x;
    if (k < c) out[dst + k] = v[q];
  }
}

__global__ void zero_u64x2_kernel(u64* p) {
  p[0] = 0;
  p[1] = 0;
}

// ----------------------------------------------------------------- merge

constexpr int kMgNT = 256;
constexpr int kMgItems = 8;
constexpr u64 kMgTile = u64(kMgNT) * kMgItems;

// Number of elements of `a` among the first `diag` outputs of the merge
// (ties: a first).
template <typename K>
__device__ __forceinline__ u64 merge_path(const K* a, u64 na, const K* b, u64 nb, u64 diag) {
  u64 lo = diag > nb ? diag - nb : 0;
  u64 hi = diag < na ? diag : na;
  while (lo < hi) {
    u64 mid = (lo + hi) >> 1;
    if (!(b[diag - 1 - mid] < a[mid])) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <typename K>
__global__ void merge_partition_kernel(const K* a, u64 na, const K* b, u64 nb, u64* parts,
                                       u64 nparts, u64 tile_len) {
  u64 t = u64(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nparts) return;
  u64 diag = t * tile_len;
  if (diag > na + nb) diag = na + nb;
  parts[t] = merge_path(a, na, b, nb, diag);
}

template <typename K>
__global__ __launch_bounds__(kMgNT) void merge_kernel(const K* a, u64 na, const K* b, u64 nb,
                                                      const u64* parts, K* out) {
  // the merged tile goes back through LDS padded by one slot per
  // kMgItems keys, so that each thread's run of kMgItems writes falls in
  // distinct banks
  __shared__ K s[kMgTile + kMgTile / kMgItems];
  const u32 tile = xcd_tile(blockIdx.x, gridDim.x);
  const u64 d0 = u64(tile) * kMgTile;
  const u64 d1 = (d0 + kMgTile) < (na + nb) ? (d0 + kMgTile) : (na + nb);
  const u64 a0 = parts[tile], a1 = parts[tile + 1];
  const u64 b0 = d0 - a0, b1 = d1 - a1;
  const u32 la = u32(a1 - a0), lb = u32(b1 - b0);
  const u32 total = la + lb;
  {
    // both slices side by side, every load issued before any is stored
    K v[kMgItems];
#pragma unroll
    for (int q = 0; q < kMgItems; ++q) {
      const u32 k = u32(q) * kMgNT + threadIdx.x;
      v[q] = k < la ? a[a0 + k] : (k < total ? b[b0 + (k - la)] : K(0));
    }
#pragma unroll
    for (int q = 0; q < kMgItems; ++q) {
      const u32 k = u32(q) * kMgNT + threadIdx.x;
      if (k < total) s[k] = v[q];
    }
  }
  __syncthreads();
  u32 diag = threadIdx.x * kMgItems;
  if (diag > total) diag = total;
  u32 ai = u32(merge_path(s, la, s + la, lb, diag));
  u32 bi = diag - ai;
  K r[kMgItems];
#pragma unroll
  for (int k = 0; k < kMgItems; ++k) {
    K v = 0;
    if (diag + k < total) {  // then ai < la or bi < lb
      bool take_a = (bi >= lb) || (ai < la && !(s[la + bi] < s[ai]));
      if (take_a) {
        v = s[ai];
        ++ai;
      } else {
        v = s[la + bi];
        ++bi;
      }
    }
    r[k] = v;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kMgItems; ++k) {
    u32 o = threadIdx.x * kMgItems + k;
    if (o < total) s[o + o / kMgItems] = r[k];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kMgItems; ++q) {
    const u32 k = u32(q) * kMgNT + threadIdx.x;
    if (k < total) out[d0 + k] = s[k + k / kMgItems];
  }
}

// Set difference by merge path, used when full has at most kUmFullPerCand
// keys per candidate (then nearly every key of full lies between two
// candidates and would be read by the select too).  The merged order of the candidates and
// full (ties: the candidate first) is cut into tiles of kUmTile positions;
// a tile loads both of its slices in one round and each thread walks
// kUmItems consecutive merged positions.  A candidate is in full exactly
// when the first key of full not yet passed equals it (the merge never
// passes a key of full that is not below the candidate).  Survivors are
// written compacted (in order) from the tile's first candidate in tmp;
// kept and distinct counts go to tile_counts and tile_uniq as in the
// select above, and a tail run is searched in the same way.
constexpr int kUmItems = 16;
constexpr u64 kUmTile = u64(kUdNT) * kUmItems;
constexpr u64 kUmFullPerCand = 1;  // the merge path is taken for nf <= n

template <typename K>
__global__ __launch_bounds__(kUdNT) __attribute__((amdgpu_waves_per_eu(sizeof(K) == 4 ? 8 : 1)))
void ud_merge_kernel(const K* cand, u64 n, const K* full, u64 nf, const u64* parts, K* tmp,
                     u32* tile_counts, u32* tile_uniq, const K* tail, u64 ntail,
                     u64* alg_bytes) {
  __shared__ u32 wsum[kUdNT / kWave];
  __shared__ K s[kUmTile + kUmTile / kUmItems];
  const u32 tile = blockIdx.x;
  const u64 d0 = u64(tile) * kUmTile;
  const u64 d1 = (d0 + kUmTile) < (n + nf) ? (d0 + kUmTile) : (n + nf);
  const u64 a0 = parts[tile], a1 = parts[tile + 1];
  const u64 b0 = d0 - a0, b1 = d1 - a1;
  const u32 la = u32(a1 - a0), lb = u32(b1 - b0);
  const u32 total = la + lb;
  // the candidate before the tile (for the first-of-run test) and the key
  // of full after it (the next unpassed key once the tile's slice is spent)
  const bool has_before = a0 > 0, has_after = b1 < nf;
  const K before = has_before ? cand[a0 - 1] : K(0);
  const K after = has_after ? full[b1] : K(0);
  {
    K v[kUmItems];
#pragma unroll
    for (int q = 0; q < kUmItems; ++q) {
      const u32 k = u32(q) * kUdNT + threadIdx.x;
      v[q] = k < la ? cand[a0 + k] : (k < total ? full[b0 + (k - la)] : K(0));
    }
#pragma unroll
    for (int q = 0; q < kUmItems; ++q) {
      const u32 k = u32(q) * kUdNT + threadIdx.x;
      if (k < total) s[k] = v[q];
    }
  }
  __syncthreads();
  u32 diag = threadIdx.x * kUmItems;
  if (diag > total) diag = total;
  u32 ai = u32(merge_path(s, la, s + la, lb, diag));
  u32 bi = diag - ai;
  bool has_prev = ai > 0 || has_before;
  K prev = ai > 0 ? s[ai - 1] : before;
  K val[kUmItems];
  u32 keep_bits = 0, nkeep = 0, uniq = 0;
  // Branch-free steps: both heads are read (at a valid index when a side
  // is spent) and selects decide; a branch per step would diverge within
  // a wave and run both sides.
#pragma unroll
  for (int k = 0; k < kUmItems; ++k) {
    const bool live = diag + k < total;  // then ai < la or bi < lb
    const bool a_left = ai < la, b_left = bi < lb;
    const K x = s[a_left ? ai : 0u];
    const K y = s[b_left ? la + bi : 0u];
    const bool take_a = live && (!b_left || (a_left && !(y < x)));
    const bool first = take_a && (!has_prev || x != prev);
    // the first key of full not yet passed: y, or the one after the tile
    const bool in_full = b_left ? (y == x) : (has_after && after == x);
    const bool keep = first && !in_full;
    val[k] = x;
    uniq += first ? 1u : 0u;
    nkeep += keep ? 1u : 0u;
    keep_bits |= keep ? (1u << k) : 0u;
    prev = take_a ? x : prev;
    has_prev = has_prev || take_a;
    ai += take_a ? 1u : 0u;
    bi += (live && !take_a) ? 1u : 0u;
  }
  // the tail: every survivor searched there, kUdLock at a time in lockstep
  const u32 tail_searched = ntail > 0 ? nkeep : 0u;
  if (ntail > 0) {
#pragma unroll
    for (int g = 0; g < kUmItems; g += kUdLock) {
      if (!((keep_bits >> g) & ((1u << kUdLock) - 1))) continue;
      const K* at[kUdLock];
#pragma unroll
      for (int j = 0; j < kUdLock; ++j) at[j] = tail;
      u64 len = ntail;
      while (len > 1) {
        const u64 half = len >> 1;
#pragma unroll
        for (int j = 0; j < kUdLock; ++j)
          if ((keep_bits >> (g + j)) & 1u) at[j] = (at[j][half] < val[g + j]) ? at[j] + half : at[j];
        len -= half;
      }
#pragma unroll
      for (int j = 0; j < kUdLock; ++j) {
        if ((keep_bits >> (g + j)) & 1u) {
          const u64 p = u64(at[j] - tail) + ((*at[j] < val[g + j]) ? 1 : 0);
          if (p < ntail && tail[p] == val[g + j]) {
            keep_bits &= ~(1u << (g + j));
            --nkeep;
          }
        }
      }
    }
  }
  static_assert(kUmTile < (u64(1) << 16), "tile counts share one word");
  u32 packed_total;
  const u32 packed = block_exclusive_scan<kUdNT>(nkeep | (uniq << 16), wsum, packed_total);
  u32 pos = packed & 0xffffu;
  const u32 kept = packed_total & 0xffffu;
  uniq = packed_total >> 16;
  // every read of s happened before the scan's barriers
#pragma unroll
  for (int k = 0; k < kUmItems; ++k)
    if (keep_bits & (1u << k)) s[pad<kUmItems>(pos++)] = val[k];
  __syncthreads();
  for (u32 k = threadIdx.x; k < kept; k += kUdNT) tmp[a0 + k] = s[pad<kUmItems>(k)];
  u32 searched = 0;
  if (alg_bytes) searched = block_sum<kUdNT>(tail_searched, wsum);
  if (threadIdx.x == 0) {
    tile_counts[tile] = kept;
    tile_uniq[tile] = uniq;
    if (alg_bytes) {
      const u64 full_b = u64(lb) * sizeof(K) < u64(uniq) * 64 ? u64(lb) * sizeof(K) : u64(uniq) * 64;
      const u64 tail_b =
          ntail * sizeof(K) < u64(searched) * 64 ? ntail * sizeof(K) : u64(searched) * 64;
      atomicAdd(reinterpret_cast<unsigned long long*>(alg_bytes),
                static_cast<unsigned long long>(u64(la + kept) * sizeof(K) + full_b + tail_b));
    }
  }
}

u64 ud_tiles(u64 n, u64 tile) { return (n + tile - 1) / tile; }
u64 mg_tiles(u64 n) { return (n + kMgTile - 1) / kMgTile; }

// The workspace of one set difference: per-tile kept and distinct counts,
// the kept counts' offsets, and the partition (two bounds per tile for the
// select, one diagonal split per tile boundary for the merge path; the
// distinct counts' prefix sum goes after the first nt + 1 entries once the
// tiles have run).  The merge path is taken when full has no more keys
// than kUmFullPerCand times the candidates (with 2 or 4 keys of full per
// candidate the merge path measured slower than the select on the
// same-generation fixpoint); the workspace is sized for the larger tile
// count of the two paths.
struct UdLayout {
  bool by_merge;
  u64 tile_keys, nt;
  u32* tile_counts;
  u32* tile_uniq;
  u64* tile_off;
  u64* part;
  char* rest;
};

UdLayout ud_layout(u64 n, u64 nf, int items, void* ws) {
  UdLayout L;
  L.by_merge = nf > 0 && nf <= kUmFullPerCand * n;
  L.tile_keys = L.by_merge ? kUmTile : u64(kUdNT) * u64(items);
  L.nt = L.by_merge ? ud_tiles(n + nf, kUmTile) : ud_tiles(n, L.tile_keys);
  char* p = static_cast<char*>(ws);
  L.tile_counts = reinterpret_cast<u32*>(p);
  p += align_up(L.nt * sizeof(u32), 256);
  L.tile_uniq = reinterpret_cast<u32*>(p);
  p += align_up(L.nt * sizeof(u32), 256);
  L.tile_off = reinterpret_cast<u64*>(p);
  p += align_up((L.nt + 1) * sizeof(u64), 256);
  L.part = reinterpret_cast<u64*>(p);
  p += align_up((2 * L.nt + 1) * sizeof(u64), 256);
  L.rest = p;
  return L;
}

}  // namespace

u64 unique_diff_workspace_bytes(u64 n) {
  // the select's smallest tile, or the merge path over at most
  // (1 + kUmFullPerCand) n keys: whichever makes more tiles
  const u64 sel = ud_tiles(n, kUdMinTile), mrg = ud_tiles((1 + kUmFullPerCand) * n, kUmTile);
  const u64 nt = sel > mrg ? sel : mrg;
  return 2 * align_up(nt * sizeof(u32), 256) + align_up((nt + 1) * sizeof(u64), 256) +
         align_up((2 * nt + 1) * sizeof(u64), 256) + scan_workspace_bytes(nt);
}

template <typename K>
hipError_t unique_diff(const K* sorted, u64 n, const K* full, u64 nf, K* tmp, K* out,
                       u64* d_counts, void* ws, hipStream_t s, LaunchTimer* timer,
                       const LearnedView<K>* model, const K* tail, u64 ntail, int items,
                       u64* lockstep_tiles) {
  zero_u64x2_kernel<<<1, 1, 0, s>>>(d_counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n == 0) return e;
  if (n >= (u64(1) << 32)) return hipErrorInvalidValue;
  if (items != 8 && items != 16) return hipErrorInvalidValue;
  const UdLayout L = ud_layout(n, nf, items, ws);
  const u64 tile_keys = L.tile_keys, nt = L.nt;
  u32* tile_counts = L.tile_counts;
  u32* tile_uniq = L.tile_uniq;
  u64* tile_off = L.tile_off;
  u64* part = L.part;
  char* p = L.rest;
  if (model && (model->keys != full || model->n != nf)) return hipErrorInvalidValue;
  // Candidates at least one per 8 keys of full leave tiles' slices short
  // enough to stream, where the model is not used; the kernel without it
  // needs fewer registers and runs more waves per SIMD.
  if (model && nf < 8 * n) model = nullptr;
  const u32 pb = u32((2 * nt + kUdNT - 1) / kUdNT);
  u64* alg = timer ? timer->device_counter(s) : nullptr;
  const LearnedView<K> lv = model ? *model : LearnedView<K>{};
  const dim3 grid = dim3(u32(nt));
  if (timer) timer->begin(K_UNIQUE_DIFF, s);
  if (L.by_merge) {
    merge_partition_kernel<K><<<dim3(u32((nt + 1 + 255) / 256)), 256, 0, s>>>(
        sorted, n, full, nf, part, nt + 1, kUmTile);
    ud_merge_kernel<K><<<grid, kUdNT, 0, s>>>(sorted, n, full, nf, part, tmp, tile_counts,
                                              tile_uniq, tail, ntail, alg);
  } else {
    if (model)
      ud_partition_kernel<K, true><<<dim3(pb), kUdNT, 0, s>>>(sorted, n, full, nf, nt,
                                                              tile_keys, part, lv);
    else
      ud_partition_kernel<K, false><<<dim3(pb), kUdNT, 0, s>>>(sorted, n, full, nf, nt,
                                                               tile_keys, part, lv);
    if (model && items == 16)
      ud_select_kernel<K, true, 16><<<grid, kUdNT, 0, s>>>(sorted, n, full, nf, tmp,
                                                            tile_counts, tile_uniq, lv, part, tail,
                                                            ntail, alg, lockstep_tiles);
    else if (model)
      ud_select_kernel<K, true, 8><<<grid, kUdNT, 0, s>>>(sorted, n, full, nf, tmp, tile_counts,
                                                           tile_uniq, lv, part, tail, ntail, alg,
                                                           lockstep_tiles);
    else if (items == 16)
      ud_select_kernel<K, false, 16><<<grid, kUdNT, 0, s>>>(sorted, n, full, nf, tmp,
                                                             tile_counts, tile_uniq, lv, part,
                                                             tail, ntail, alg, lockstep_tiles);
    else
      ud_select_kernel<K, false, 8><<<grid, kUdNT, 0, s>>>(sorted, n, full, nf, tmp,
                                                            tile_counts, tile_uniq, lv, part, tail,
                                                            ntail, alg, lockstep_tiles);
  }
  // the tiles count their own bytes (above); without a device counter only
  // the candidate reads are known here
  if (timer) timer->end(K_UNIQUE_DIFF, s, alg ? 0 : n * sizeof(K), alg);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_u32_u64(tile_counts, nt, tile_off, d_counts, p, s);
  if (e != hipSuccess) return e;
  // the distinct count: a prefix sum whose total is all that is kept (after
  // the merge path's splits, which the gather still reads)
  e = scan_u32_u64(tile_uniq, nt, part + nt + 1, d_counts + 1, p, s);
  if (e != hipSuccess || !out) return e;
  ud_gather_kernel<K><<<grid, kUdNT, 0, s>>>(tmp, tile_counts, tile_off, tile_keys,
                                             L.by_merge ? part : nullptr, out);
  return hipGetLastError();
}

template <typename K>
hipError_t unique_diff_gather(const K* tmp, u64 n, u64 nf, const void* ws, K* out, hipStream_t s,
                              int items) {
  if (n == 0) return hipSuccess;
  if (n >= (u64(1) << 32) || (items != 8 && items != 16)) return hipErrorInvalidValue;
  const UdLayout L = ud_layout(n, nf, items, const_cast<void*>(ws));
  ud_gather_kernel<K><<<dim3(u32(L.nt)), kUdNT, 0, s>>>(tmp, L.tile_counts, L.tile_off,
                                                        L.tile_keys, L.by_merge ? L.part : nullptr,
                                                        out);
  return hipGetLastError();
}

u64 merge_workspace_bytes(u64 na, u64 nb) {
  return align_up((mg_tiles(na + nb) + 1) * sizeof(u64), 256);
}

template <typename K>
hipError_t merge(const K* a, u64 na, const K* b, u64 nb, K* out, void* ws, hipStream_t s,
                 LaunchTimer* timer) {
  const u64 n = na + nb;
  if (n == 0) return hipSuccess;
  const u64 nt = mg_tiles(n);
  if (nt >= (u64(1) << 31)) return hipErrorInvalidValue;
  u64* parts = static_cast<u64*>(ws);
  const u64 nparts = nt + 1;
  merge_partition_kernel<K><<<dim3(u32((nparts + 255) / 256)), 256, 0, s>>>(a, na, b, nb, parts,
                                                                           nparts, kMgTile);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (timer) timer->begin(K_MERGE, s);
  merge_kernel<K><<<dim3(u32(nt)), kMgNT, 0, s>>>(a, na, b, nb, parts, out);
  if (timer) timer->end(K_MERGE, s, 2 * n * sizeof(K));
  return hipGetLastError();
}

template hipError_t unique_diff<u32>(const u32*, u64, const u32*, u64, u32*, u32*, u64*, void*,
                                     hipStream_t, LaunchTimer*, const LearnedView<u32>*,
                                     const u32*, u64, int, u64*);
template hipError_t unique_diff<u64>(const u64*, u64, const u64*, u64, u64*, u64*, u64*, void*,
                                     hipStream_t, LaunchTimer*, const LearnedView<u64>*,
                                     const u64*, u64, int, u64*);
template hipError_t unique_diff_gather<u32>(const u32*, u64, u64, const void*, u32*,
                                            hipStream_t, int);
template hipError_t unique_diff_gather<u64>(const u64*, u64, u64, const void*, u64*,
                                            hipStream_t, int);
template hipError_t merge<u32>(const u32*, u64, const u32*, u64, u32*, void*, hipStream_t,
                               LaunchTimer*);
template hipError_t merge<u64>(const u64*, u64, const u64*, u64, u64*, void*, hipStream_t,
                               LaunchTimer*);

}  // namespace hl
