// Binary join of an outer pair array against an inner HISA (Section 5.1,
// "Implementing Joins", Algorithm 3): every outer tuple hashes its join
// column, finds the start of the matching run of the inner sorted array,
// and scans the run, emitting one projected (and filtered) pair per inner
// tuple.  Multi-atom bodies run one such join per atom with the
// intermediate result materialised (Section 5.2).
//
// GPU shape.  Algorithm 3 gives one thread per outer tuple, so a hub key
// with a long run keeps one lane busy while its wave idles (the imbalance
// Section 5.2 describes for nested joins).  Here the join is three passes:
//   probe   one lane per outer tuple: (run start, run length);
//   scan    exclusive prefix of the lengths = output offsets;
//   expand  output positions are split evenly over workgroups by a merge
//           path of the offsets against the output index (load-balanced
//           search), so every lane emits about the same number of pairs
//           whatever the run lengths, with coalesced reads of each run and
//           coalesced writes.
// When the outer is grouped by the column it carries into the output,
// consecutive outer tuples produce outputs that share that column, and the
// same output often comes from several of them (Reach: one target reached
// through several middle nodes).  The expand can then drop the repeats
// within each tile in an LDS hash set before they are written, so the sort
// that follows moves fewer keys; the set of outputs is unchanged.
#include "device.hpp"
#include "kernels.hpp"

namespace hl {

namespace {

constexpr int kNT = 256;
constexpr int kItems = 8;
constexpr u64 kTile = u64(kNT) * kItems;

// Linear probing from slot `slot`, whose entry `sl` has been read already.
__device__ __forceinline__ bool hisa_resolve(const Slot* table, u64 cap, u32 key, u64 slot,
                                             Slot sl, u32& start, u32& len) {
  for (u64 probe = 0; probe < cap; ++probe) {
    if (probe > 0) sl = table[slot];
    if (sl.w0 == 0) return false;
    if (u32(sl.w0) == key) {
      len = u32(sl.w0 >> 32);
      start = u32(sl.w1);
      return true;
    }
    slot = (slot + 1 == cap) ? 0 : slot + 1;
  }
  return false;
}

__device__ __forceinline__ bool hisa_find(const Slot* table, u64 cap, u32 key, u32& start,
                                          u32& len) {
  const u64 slot = slot_of(key, cap);
  return hisa_resolve(table, cap, key, slot, table[slot], start, len);
}

// Value number src of (c0, c1, inner's other column); 3 is the constant 0
// (the second column of a unary relation).
template <typename K>
__device__ __forceinline__ K pick(int src, K c0, K c1, K o) {
  return src == 0 ? c0 : (src == 1 ? c1 : (src == 2 ? o : K(0)));
}

// kProbeItems outer tuples per lane, in rounds of kNT consecutive tuples
// per block (64 per wave): every round's outer loads are issued first, then
// every round's probes, then the writes, so a wave keeps several
// independent memory accesses in flight.  Outer arrays are sorted on (or
// grouped by) their first column, so neighbouring tuples often share the
// join key: only the first lane of each run of equal keys within a wave
// probes, and the run's other lanes take its result by a wave shuffle.
constexpr int kProbeItems = 4;

template <typename K>
__global__ __launch_bounds__(kNT) void probe_kernel(const K* outer, u64 n, int outer_col, int w,
                                                    const Slot* table, u64 cap, u32* start,
                                                    u32* len) {
  const K mask = (K(1) << w) - 1;
  const u64 i0 = u64(blockIdx.x) * (kNT * kProbeItems) + threadIdx.x;
  const int lane = lane_id();
  // every load of a phase is issued before any of its values is used (work
  // on a value inside its load's branch would wait for that load first)
  K kv[kProbeItems];
#pragma unroll
  for (int r = 0; r < kProbeItems; ++r) {
    const u64 i = i0 + u64(r) * kNT;
    kv[r] = i < n ? outer[i] : K(0);
  }
  u32 jc[kProbeItems];
#pragma unroll
  for (int r = 0; r < kProbeItems; ++r) jc[r] = outer_col == 0 ? u32(kv[r] >> w) : u32(kv[r] & mask);
  // a wave's first lane always probes; any other lane probes when its key
  // differs from the lane below.  The leaders' home slots are read together,
  // then collisions are followed one round at a time.
  u64 lm[kProbeItems], home[kProbeItems];
  bool lead[kProbeItems];
#pragma unroll
  for (int r = 0; r < kProbeItems; ++r) {
    const u64 i = i0 + u64(r) * kNT;
    const u32 below = __shfl_up(jc[r], 1, kWave);
    lead[r] = i < n && (lane == 0 || jc[r] != below);
    lm[r] = ballot(lead[r]);
    home[r] = slot_of(jc[r], cap);
  }
  Slot sl[kProbeItems];
#pragma unroll
  for (int r = 0; r < kProbeItems; ++r) sl[r] = (lead[r] && cap > 0) ? table[home[r]] : Slot{0, 0};
  u32 st[kProbeItems], ln[kProbeItems];
#pragma unroll
  for (int r = 0; r < kProbeItems; ++r) {
    st[r] = ln[r] = 0;
    if (lead[r] && !hisa_resolve(table, cap, jc[r], home[r], sl[r], st[r], ln[r])) ln[r] = 0;
  }
#pragma unroll
  for (int r = 0; r < kProbeItems; ++r) {
    const u64 i = i0 + u64(r) * kNT;
    // the leader of this lane's run: highest leader lane at or below it
    const u64 upto = lm[r] & ((lane == 63) ? ~u64(0) : ((u64(2) << lane) - 1));
    const int src = upto ? 63 - __clzll((long long)upto) : lane;
    const u32 s0 = __shfl(st[r], src, kWave);
    const u32 l0 = __shfl(ln[r], src, kWave);
    if (i < n) {
      start[i] = s0;
      len[i] = l0;
    }
  }
}

template <typename K>
__global__ __launch_bounds__(kNT) void probe_learned_kernel(const K* outer, u64 n, int outer_col,
                                                            int w, LearnedView<K> lv, u32* start,
                                                            u32* len) {
  const K mask = (K(1) << w) - 1;
  const u64 i0 = u64(blockIdx.x) * (kNT * kProbeItems) + threadIdx.x;
  const int lane = lane_id();
  K kv[kProbeItems];
#pragma unroll
  for (int r = 0; r < kProbeItems; ++r) {
    const u64 i = i0 + u64(r) * kNT;
    kv[r] = i < n ? outer[i] : K(0);
  }
  u32 jc[kProbeItems];
#pragma unroll
  for (int r = 0; r < kProbeItems; ++r) jc[r] = outer_col == 0 ? u32(kv[r] >> w) : u32(kv[r] & mask);
#pragma unroll
  for (int r = 0; r < kProbeItems; ++r) {
    const u64 i = i0 + u64(r) * kNT;
    const u32 below = __shfl_up(jc[r], 1, kWave);
    const bool leader = i < n && (lane == 0 || jc[r] != below);
    const u64 lm = ballot(leader);
    u32 st = 0, ln = 0;
    if (leader) {
      st = lm_lower_bound(lv, K(jc[r]) << w);
      // the run's end: gallop forward from its start (runs are short, so
      // this stays within a cache line or two of the start), then bisect
      if (st < lv.n && K(lv.keys[st] >> w) == K(jc[r])) {
        u64 good = st, step = 1;  // keys[good] is in the run
        while (good + step < lv.n && K(lv.keys[good + step] >> w) == K(jc[r])) {
          good += step;
          step <<= 1;
        }
        u64 lo = good + 1, hi = (good + step < lv.n) ? good + step : lv.n;  // end in [lo, hi]
        while (lo < hi) {
          const u64 mid = (lo + hi) >> 1;
          if (K(lv.keys[mid] >> w) == K(jc[r])) lo = mid + 1;
          else hi = mid;
        }
        ln = u32(lo - st);
      }
    }
    const u64 upto = lm & ((lane == 63) ? ~u64(0) : ((u64(2) << lane) - 1));
    const int src = upto ? 63 - __clzll((long long)upto) : lane;
    st = __shfl(st, src, kWave);
    ln = __shfl(ln, src, kWave);
    if (i < n) {
      start[i] = ln ? st : 0;
      len[i] = ln;
    }
  }
}

// Merged order of outer tuple i (key off[i]) and output j (key j): the
// outer tuple comes first when off[i] <= j.  Returns how many outer tuples
// are among the first `diag` merged items.
__device__ __forceinline__ u64 lbs_path(const u64* off, u64 na, u64 nb, u64 diag) {
  u64 lo = diag > nb ? diag - nb : 0;
  u64 hi = diag < na ? diag : na;
  while (lo < hi) {
    u64 mid = (lo + hi) >> 1;
    if (off[mid] <= diag - 1 - mid) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ void lbs_partition_kernel(const u64* off, u64 na, u64 nb, u64* parts, u64 nparts,
                                     u64 tile) {
  const u64 t = u64(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nparts) return;
  u64 diag = t * tile;
  if (diag > na + nb) diag = na + nb;
  parts[t] = lbs_path(off, na, nb, diag);
}

// Block-level compaction of filtered outputs: survivors are gathered in LDS
// in order, then the block claims one range of the output with a single
// atomic and writes it coalesced.  (Order between blocks is arbitrary; the
// new tuples are sorted afterwards.)
template <typename K>
struct Compactor {
  K* buf;         // LDS, kTile entries
  u32* counter;   // LDS
  u32* wsum;      // LDS, kNT / 64
  __device__ void add(K v, bool keep) {
    u32 tot;
    u32 pos = block_exclusive_scan<kNT>(keep ? 1u : 0u, wsum, tot);
    const u32 base = *counter;
    if (keep) buf[base + pos] = v;
    __syncthreads();
    if (threadIdx.x == 0) *counter = base + tot;
    __syncthreads();
  }
  __device__ void flush(K* out, u64* cursor, u64* s_base) {
    const u32 n = *counter;
    if (threadIdx.x == 0)
      *s_base = n ? atomicAdd(reinterpret_cast<unsigned long long*>(cursor),
                              (unsigned long long)n)
                  : 0;
    __syncthreads();
    const u64 base = *s_base;
    for (u32 k = threadIdx.x; k < n; k += kNT) out[base + k] = buf[k];
  }
};

// Outputs of one expand tile, deduplicated in an LDS hash set of SLOTS
// keys (twice the tile) with linear probing.  A tile emits at most half
// that many keys, so the set is at most half full and every insertion finds
// its key or an empty slot.  The all-ones key marks an empty slot; that one
// key value is never dropped here (the sort and unique that follow remove
// its repeats).
template <u32 SLOTS, typename K>
__device__ __forceinline__ bool first_in_tile(K* set, K v) {
  const K empty = ~K(0);
  if (v == empty) return true;
  u32 h = mix32(u32(v) ^ u32(u64(v) >> 32)) & (SLOTS - 1);
  for (u32 probe = 0; probe < SLOTS; ++probe) {
    K prev;
    if constexpr (sizeof(K) == 8)
      prev = K(atomicCAS(reinterpret_cast<unsigned long long*>(set + h),
                         (unsigned long long)empty, (unsigned long long)v));
    else
      prev = K(atomicCAS(reinterpret_cast<unsigned int*>(set + h), (unsigned int)empty,
                         (unsigned int)v));
    if (prev == empty) return true;
    if (prev == v) return false;
    h = (h + 1) & (SLOTS - 1);
  }
  return true;
}

// How an expand turns (outer tuple, inner tuple) into an output: binary
// relations (a pair and the inner's other column), or relations of arity up
// to 4 (WideSpec: any columns of either side).
template <typename K>
struct PairGather {
  JoinSpec js;
  __device__ bool filtered() const { return js.fa >= 0 || js.ea >= 0 || js.dd; }
  __device__ bool dedup() const { return js.dd != 0; }
  __device__ K operator()(K ok, K ik, bool& pass) const {
    const K mask = (K(1) << js.w) - 1;
    const K c0 = ok >> js.w, c1 = ok & mask;
    const K o = ik & mask;
    const K x = pick(js.src0, c0, c1, o), y = pick(js.src1, c0, c1, o);
    pass = (js.fa < 0 || pick(js.fa, c0, c1, o) != pick(js.fb, c0, c1, o)) &&
           (js.ea < 0 || pick(js.ea, c0, c1, o) == pick(js.eb, c0, c1, o));
    return (x << js.w) | y;
  }
};

template <typename K>
struct WideGather {
  WideSpec ws;
  __device__ bool filtered() const { return ws.nf > 0 || ws.ne > 0; }
  __device__ bool dedup() const { return false; }
  __device__ K operator()(K ok, K ik, bool& pass) const { return wide_gather(ok, ik, ws, pass); }
};

// ITEMS outputs per thread: a tile of kNT * ITEMS outputs and outer tuples.
// An inner relation kept as two sorted runs (a large run and a short tail
// beside it) is joined in one pass: entries i < n_split of off/start are
// runs of outer tuple i in `inner`, entries n_split + i runs of the same
// outer tuple in `inner2` (n_split == n_outer when there is one run).
template <typename K, int ITEMS, typename G>
__global__ __launch_bounds__(kNT) void expand_kernel(const K* outer, u64 n_outer, const u64* off,
                                                     const u32* start, const K* inner,
                                                     const K* inner2, u64 n_split, u64 total,
                                                     G g, const u64* parts, u64 tile0, K* out,
                                                     u64* cursor) {
  constexpr u64 kTile = u64(kNT) * ITEMS;
  constexpr int kItems = ITEMS;
  constexpr u32 kDedupSlots = 2 * u32(kTile);
  // Offsets of the tile's outer tuples relative to its first output b0: the
  // merge path puts every one of them in [b0, b1], so 32 bits hold them.
  // s_pool holds them (la words), the owner of each of the tile's outputs
  // right after them (lb words; la + lb <= kTile) and, from kTile on, each
  // run's position base (la + 1 words: entry 0 for the run carried in from
  // before the tile, entry j for outer tuple a0 + j - 1); after the block
  // scan below (once all are no longer read) it holds the surviving outputs
  // instead.  Output k of the tile owned by outer tuple i reads the inner
  // tuple at base + k (mod 2^32; inner positions are 32-bit).
  __shared__ u32 s_pool[2 * kTile + 1];
  static_assert(sizeof(K) * kTile <= sizeof(u32) * 2 * kTile, "survivors fit the pool");
  u32* s_off = s_pool;
  u32* s_pbase = s_pool + kTile;
  // tiles tile0 .. tile0 + gridDim.x - 1; unfiltered outputs are written
  // relative to the first output of tile0
  const u64 tile = tile0 + blockIdx.x;
  const u64 obase = tile0 * kTile - parts[tile0];
  const u64 d0 = tile * kTile;
  const u64 dend = n_outer + total;
  const u64 d1 = (d0 + kTile) < dend ? (d0 + kTile) : dend;
  const u64 a0 = parts[tile], a1 = parts[tile + 1];
  const u64 b0 = d0 - a0, b1 = d1 - a1;
  const u32 la = u32(a1 - a0), lb = u32(b1 - b0);
  u32* s_owner = s_pool + la;
  {
    // the tile's outer tuples (at most kTile) and the run carried in, every
    // load issued before any is stored.  Only the low words of the 64-bit
    // offsets are read: the tile's relative offsets fit 32 bits, and a
    // 64-bit load whose high half is dead lets the compiler reuse that half
    // while the load is in flight, which costs a wait per load.
    const u32* off_lo = reinterpret_cast<const u32*>(off);
    u32 o_off[kItems], o_start[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const u32 k = u32(r) * kNT + threadIdx.x;
      const u64 i = a0 + k;
      o_off[r] = k < la ? off_lo[2 * i] : u32(b0);
      o_start[r] = k < la ? start[i] : 0u;
    }
    const bool carry = threadIdx.x == 0 && a0 > 0;
    const u64 c_off = carry ? off[a0 - 1] : b0;
    const u32 c_start = carry ? start[a0 - 1] : 0u;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const u32 k = u32(r) * kNT + threadIdx.x;
      if (k < la) {
        const u32 rel = o_off[r] - u32(b0);
        s_off[k] = rel;
        s_pbase[k + 1] = o_start[r] - rel;
      }
    }
    if (threadIdx.x == 0) s_pbase[0] = c_start + u32(b0 - c_off);
  }
  __syncthreads();
  // serial merge of this thread's slice of the tile's merged sequence
  {
    const u32 tot = la + lb;
    u32 diag = threadIdx.x * kItems;
    if (diag > tot) diag = tot;
    u32 lo = diag > lb ? diag - lb : 0;
    u32 hi = diag < la ? diag : la;
    while (lo < hi) {
      u32 mid = (lo + hi) >> 1;
      if (s_off[mid] <= diag - 1 - mid) lo = mid + 1;
      else hi = mid;
    }
    u32 ai = lo, bi = diag - lo;
    for (int k = 0; k < kItems && diag + k < tot; ++k) {
      if (ai < la && (bi >= lb || s_off[ai] <= bi)) {
        ++ai;
      } else {
        s_owner[bi] = ai;  // run ai: outer tuple a0 + ai - 1
        ++bi;
      }
    }
  }
  __syncthreads();
  const bool filtered = g.filtered();
  K* s_keep = reinterpret_cast<K*>(s_pool);
  __shared__ u32 s_wsum[kNT / kWave];
  __shared__ u64 s_base;
  // the dedup set lives in dynamic LDS, sized at launch only when js.dd
  extern __shared__ __align__(16) unsigned char s_dyn[];
  K* dset = reinterpret_cast<K*>(s_dyn);
  if (g.dedup())
    for (u32 k = threadIdx.x; k < kDedupSlots; k += kNT) dset[k] = ~K(0);
  if (g.dedup()) __syncthreads();
  // each thread's kItems outputs (strided, so reads of each inner run and
  // the unfiltered writes are coalesced): first every owner and position
  // from LDS, then every load, then the outputs (the gather's branches on
  // the join's columns would otherwise keep each output's loads from
  // overlapping the next one's)
  u32 own[kItems], ipos[kItems];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const u32 k = u32(r) * kNT + threadIdx.x;
    const u32 j = k < lb ? s_owner[k] : 0u;
    own[r] = u32(a0) + j - 1;  // wraps only for the unused j = 0 of tile 0
    ipos[r] = s_pbase[j] + k;
  }
  // the outer tuple from global memory (consecutive outputs share it, so it
  // is a cache hit; keeping it out of LDS leaves room for more workgroups
  // per CU), read beside the inner tuple
  K okv[kItems], ikv[kItems];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const u32 k = u32(r) * kNT + threadIdx.x;
    okv[r] = 0;
    ikv[r] = 0;
    if (k < lb) {
      const u64 i = own[r];
      okv[r] = outer[i < n_split ? i : i - n_split];
      ikv[r] = (i < n_split ? inner : inner2)[ipos[r]];
    }
  }
  K v[kItems];
  u32 keep = 0;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const u32 k = u32(r) * kNT + threadIdx.x;
    v[r] = 0;
    if (k < lb) {
      bool pass;
      v[r] = g(okv[r], ikv[r], pass);
      if (pass) keep |= 1u << r;
    }
  }
  if (!filtered) {
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const u32 k = u32(r) * kNT + threadIdx.x;
      if (k < lb) out[b0 + k - obase] = v[r];
    }
    return;
  }
  if (g.dedup()) {
#pragma unroll
    for (int r = 0; r < kItems; ++r)
      if ((keep >> r) & 1u)
        if (!first_in_tile<kDedupSlots>(dset, v[r])) keep &= ~(1u << r);
  }
  // one block scan places every survivor of the tile in LDS, then one
  // atomic claims the tile's output range
  u32 tot;
  u32 pos = block_exclusive_scan<kNT>(u32(__popc(keep)), s_wsum, tot);
#pragma unroll
  for (int r = 0; r < kItems; ++r)
    if ((keep >> r) & 1u) s_keep[pos++] = v[r];
  if (threadIdx.x == 0)
    s_base = tot ? atomicAdd(reinterpret_cast<unsigned long long*>(cursor),
                             (unsigned long long)tot)
                 : 0;
  __syncthreads();
  const u64 ob = s_base;
  for (u32 k = threadIdx.x; k < tot; k += kNT) out[ob + k] = s_keep[k];
}

template <typename K>
__global__ __launch_bounds__(kNT) void project_kernel(const K* in, u64 n, JoinSpec js, K* out,
                                                      u64* cursor) {
  __shared__ K s_keep[kTile];
  __shared__ u32 s_count;
  __shared__ u32 s_wsum[kNT / kWave];
  __shared__ u64 s_base;
  const bool filtered = js.fa >= 0 || js.ea >= 0;
  const K mask = (K(1) << js.w) - 1;
  const u64 t0 = u64(blockIdx.x) * kTile;
  Compactor<K> cmp{s_keep, &s_count, s_wsum};
  if (threadIdx.x == 0) s_count = 0;
  __syncthreads();
  for (u32 kk = 0; kk < kTile; kk += kNT) {
    const u64 i = t0 + kk + threadIdx.x;
    bool keep = false;
    K v = 0;
    if (i < n) {
      const K k = in[i];
      const K c0 = k >> js.w, c1 = k & mask;
      const K x = pick(js.src0, c0, c1, K(0)), y = pick(js.src1, c0, c1, K(0));
      v = (x << js.w) | y;
      keep = (js.fa < 0 || pick(js.fa, c0, c1, K(0)) != pick(js.fb, c0, c1, K(0))) &&
             (js.ea < 0 || pick(js.ea, c0, c1, K(0)) == pick(js.eb, c0, c1, K(0)));
    }
    if (filtered) cmp.add(v, keep);
    else if (i < n) out[i] = v;
  }
  if (filtered) cmp.flush(out, cursor, &s_base);
}

// ------------------------------------------------------ nested joins
// The paper's nested evaluation of a two-join body (Section 5.2), kept as
// an ablation of the materialised form above: one thread per outer tuple
// walks the run of its first join and, for every tuple of it, the run of
// the second join.  A first pass counts each thread's kept outputs, a scan
// turns the counts into offsets, and a second pass writes them.
struct NestedSide {
  const void* inner;
  const Slot* table;  // hash index, or null: probe through the learned view
  u64 cap;
  JoinSpec js;
};

template <typename K>
__device__ __forceinline__ void nested_run(const NestedSide& s, const LearnedView<K>& lv, u32 jc,
                                           int w, u64& start, u64& len) {
  start = 0;
  len = 0;
  if (s.table) {
    u32 st = 0, ln = 0;
    if (hisa_find(s.table, s.cap, jc, st, ln)) {
      start = st;
      len = ln;
    }
    return;
  }
  const u32 st = lm_lower_bound(lv, K(jc) << w);
  if (st >= lv.n || K(lv.keys[st] >> w) != K(jc)) return;
  const K next = (K(jc) + 1) << w;
  const u32 en = next == 0 ? u32(lv.n) : lm_lower_bound(lv, next);
  start = st;
  len = en - st;
}

template <typename K, bool kWrite>
__global__ __launch_bounds__(kNT) void nested_kernel(const K* outer, u64 n, NestedSide a,
                                                     LearnedView<K> la, NestedSide b,
                                                     LearnedView<K> lb, u32* count,
                                                     const u64* off, K* out, u32* too_many) {
  const u64 i = u64(blockIdx.x) * kNT + threadIdx.x;
  if (i >= n) return;
  const int w = a.js.w;
  const K mask = (K(1) << w) - 1;
  const K* ia = static_cast<const K*>(a.inner);
  const K* ib = static_cast<const K*>(b.inner);
  const K k = outer[i];
  const K c0 = k >> w, c1 = k & mask;
  u64 sa, na;
  nested_run(a, la, u32(a.js.outer_col == 0 ? c0 : c1), w, sa, na);
  u64 pos = kWrite ? off[i] : 0;
  u64 kept = 0;
  for (u64 x = 0; x < na; ++x) {
    const K oa = ia[sa + x] & mask;
    if (!((a.js.fa < 0 || pick(a.js.fa, c0, c1, oa) != pick(a.js.fb, c0, c1, oa)) &&
          (a.js.ea < 0 || pick(a.js.ea, c0, c1, oa) == pick(a.js.eb, c0, c1, oa))))
      continue;
    const K d0 = pick(a.js.src0, c0, c1, oa), d1 = pick(a.js.src1, c0, c1, oa);
    u64 sb, nb;
    nested_run(b, lb, u32(b.js.outer_col == 0 ? d0 : d1), w, sb, nb);
    for (u64 y = 0; y < nb; ++y) {
      const K ob = ib[sb + y] & mask;
      if (!((b.js.fa < 0 || pick(b.js.fa, d0, d1, ob) != pick(b.js.fb, d0, d1, ob)) &&
            (b.js.ea < 0 || pick(b.js.ea, d0, d1, ob) == pick(b.js.eb, d0, d1, ob))))
        continue;
      if (kWrite) out[pos++] = (pick(b.js.src0, d0, d1, ob) << w) | pick(b.js.src1, d0, d1, ob);
      else ++kept;
    }
  }
  if (!kWrite) {
    if (kept > 0xFFFFFFFFull) {
      atomicOr(too_many, 1u);  // the counts are 32-bit: the caller fails
      kept = 0;
    }
    count[i] = u32(kept);
  }
}

u64 tiles_of(u64 n) { return (n + kTile - 1) / kTile; }

}  // namespace

template <typename K>
hipError_t join_probe(const K* outer, u64 n, const JoinSpec& js, const Slot* table, u64 cap,
                      u32* start, u32* len, hipStream_t s, LaunchTimer* timer) {
  if (n == 0) return hipSuccess;
  if (cap == 0 || cap > (u64(1) << 32) || js.outer_col < 0 || js.outer_col > 1)
    return hipErrorInvalidValue;
  const u64 blocks = (n + kNT * kProbeItems - 1) / (kNT * kProbeItems);
  if (blocks >= (u64(1) << 31)) return hipErrorInvalidValue;
  if (timer) timer->begin(K_JOIN_PROBE, s);
  probe_kernel<K><<<dim3(u32(blocks)), kNT, 0, s>>>(outer, n, js.outer_col, js.w, table, cap,
                                                    start, len);
  if (timer) timer->end(K_JOIN_PROBE, s, n * (sizeof(K) + sizeof(Slot) + 2 * sizeof(u32)));
  return hipGetLastError();
}

template <typename K>
hipError_t join_probe_learned(const K* outer, u64 n, const JoinSpec& js,
                              const LearnedView<K>& lv, u32* start, u32* len, hipStream_t s,
                              LaunchTimer* timer) {
  if (n == 0) return hipSuccess;
  if (js.outer_col < 0 || js.outer_col > 1 || lv.n >= (u64(1) << 32)) return hipErrorInvalidValue;
  const u64 blocks = (n + kNT * kProbeItems - 1) / (kNT * kProbeItems);
  if (blocks >= (u64(1) << 31)) return hipErrorInvalidValue;
  if (timer) timer->begin(K_JOIN_PROBE, s);
  probe_learned_kernel<K><<<dim3(u32(blocks)), kNT, 0, s>>>(outer, n, js.outer_col, js.w, lv,
                                                            start, len);
  if (timer) timer->end(K_JOIN_PROBE, s, n * (sizeof(K) + 2 * sizeof(u32)));
  return hipGetLastError();
}

bool join_items_ok(int items) { return items == 4 || items == 8 || items == 16; }

u64 join_tile_outputs(int items) { return u64(kNT) * u64(items); }

u64 join_tiles(u64 n_outer, u64 total, int items) {
  const u64 t = join_tile_outputs(items);
  return (n_outer + total + t - 1) / t;
}

u64 join_parts(u64 n_outer, u64 total, int items) { return join_tiles(n_outer, total, items) + 1; }

hipError_t join_partition(const u64* off, u64 n_outer, u64 total, u64* parts, hipStream_t s,
                          int items) {
  if (total == 0) return hipSuccess;
  if (n_outer >= (u64(1) << 32) || !join_items_ok(items)) return hipErrorInvalidValue;
  const u64 nt = join_tiles(n_outer, total, items);
  if (nt >= (u64(1) << 31)) return hipErrorInvalidValue;
  const u64 nparts = nt + 1;
  lbs_partition_kernel<<<dim3(u32((nparts + 255) / 256)), 256, 0, s>>>(
      off, n_outer, total, parts, nparts, join_tile_outputs(items));
  return hipGetLastError();
}

template <typename K>
hipError_t join_expand_tiles(const K* outer, u64 n_outer, const u64* off, const u32* start,
                             const K* inner, u64 total, const JoinSpec& js, const u64* parts,
                             u64 tile0, u64 tiles, K* out, u64* cursor, hipStream_t s,
                             LaunchTimer* timer, int items, const K* inner2, u64 n_split) {
  if (total == 0 || tiles == 0) return hipSuccess;
  if (!join_items_ok(items)) return hipErrorInvalidValue;
  const u64 nt = join_tiles(n_outer, total, items);
  if (n_outer >= (u64(1) << 32) || tile0 + tiles > nt || tiles >= (u64(1) << 31))
    return hipErrorInvalidValue;
  if (timer) timer->begin(K_JOIN_EXPAND, s);
  // the dedup set (2 slots per tile output) lives in dynamic LDS
  const size_t dyn = js.dd ? 2 * join_tile_outputs(items) * sizeof(K) : 0;
  const dim3 grid = dim3(u32(tiles));
  const PairGather<K> g{js};
  if (!inner2 || n_split > n_outer) {
    inner2 = inner;
    n_split = n_outer;
  }
  if (items == 4)
    expand_kernel<K, 4><<<grid, kNT, dyn, s>>>(outer, n_outer, off, start, inner, inner2,
                                               n_split, total, g, parts, tile0, out, cursor);
  else if (items == 16)
    expand_kernel<K, 16><<<grid, kNT, dyn, s>>>(outer, n_outer, off, start, inner, inner2,
                                                n_split, total, g, parts, tile0, out, cursor);
  else
    expand_kernel<K, 8><<<grid, kNT, dyn, s>>>(outer, n_outer, off, start, inner, inner2,
                                               n_split, total, g, parts, tile0, out, cursor);
  // by definition: each inner tuple of a matched run read once, each output
  // written once, each outer tuple with its offset and run start read once
  // (apportioned to the launch's share of the tiles)
  if (timer) {
    const double f = double(tiles) / double(nt);
    timer->end(K_JOIN_EXPAND, s,
               u64(f * double(2 * total * sizeof(K) +
                              n_outer * (sizeof(K) + sizeof(u64) + sizeof(u32)))));
  }
  return hipGetLastError();
}

template <typename K>
hipError_t join_expand(const K* outer, u64 n_outer, const u64* off, const u32* start,
                       const K* inner, u64 total, const JoinSpec& js, u64* parts, K* out,
                       u64* cursor, hipStream_t s, LaunchTimer* timer, int items,
                       const K* inner2, u64 n_split) {
  hipError_t e = join_partition(off, n_outer, total, parts, s, items);
  if (e != hipSuccess || total == 0) return e;
  return join_expand_tiles<K>(outer, n_outer, off, start, inner, total, js, parts, 0,
                              join_tiles(n_outer, total, items), out, cursor, s, timer, items,
                              inner2, n_split);
}

template <typename K>
hipError_t wide_expand_tiles(const K* outer, u64 n_outer, const u64* off, const u32* start,
                             const K* inner, u64 total, const WideSpec& ws, const u64* parts,
                             u64 tile0, u64 tiles, K* out, u64* cursor, hipStream_t s,
                             LaunchTimer* timer) {
  if (total == 0 || tiles == 0) return hipSuccess;
  if (!wide_spec_ok(ws)) return hipErrorInvalidValue;
  const u64 nt = join_tiles(n_outer, total, 8);
  if (n_outer >= (u64(1) << 32) || tile0 + tiles > nt || tiles >= (u64(1) << 31))
    return hipErrorInvalidValue;
  if (timer) timer->begin(K_JOIN_EXPAND, s);
  expand_kernel<K, 8><<<dim3(u32(tiles)), kNT, 0, s>>>(outer, n_outer, off, start, inner, inner,
                                                       n_outer, total, WideGather<K>{ws}, parts,
                                                       tile0, out, cursor);
  if (timer) {
    const double f = double(tiles) / double(nt);
    timer->end(K_JOIN_EXPAND, s,
               u64(f * double(2 * total * sizeof(K) +
                              n_outer * (sizeof(K) + sizeof(u64) + sizeof(u32)))));
  }
  return hipGetLastError();
}

template <typename K>
hipError_t project(const K* in, u64 n, const JoinSpec& js, K* out, u64* cursor, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const u64 blocks = tiles_of(n);
  if (blocks >= (u64(1) << 31)) return hipErrorInvalidValue;
  project_kernel<K><<<dim3(u32(blocks)), kNT, 0, s>>>(in, n, js, out, cursor);
  return hipGetLastError();
}

template <typename K>
hipError_t join_nested(const K* outer, u64 n, const NestedJoin<K>& nj, u32* count, u64* off,
                       u64* d_total, u32* too_many, void* scan_ws, K* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const u64 blocks = (n + kNT - 1) / kNT;
  if (blocks >= (u64(1) << 31) || n >= (u64(1) << 32)) return hipErrorInvalidValue;
  for (int q = 0; q < 2; ++q) {
    const JoinSpec& js = nj.js[q];
    if (!nj.inner[q] || (!nj.table[q] && !nj.lv[q].keys) || js.outer_col < 0 ||
        js.outer_col > 1)
      return hipErrorInvalidValue;
  }
  NestedSide a{nj.inner[0], nj.table[0], nj.cap[0], nj.js[0]};
  NestedSide b{nj.inner[1], nj.table[1], nj.cap[1], nj.js[1]};
  if (!out) {
    nested_kernel<K, false><<<dim3(u32(blocks)), kNT, 0, s>>>(outer, n, a, nj.lv[0], b, nj.lv[1],
                                                              count, nullptr, nullptr, too_many);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return scan_u32_u64(count, n, off, d_total, scan_ws, s);
  }
  nested_kernel<K, true><<<dim3(u32(blocks)), kNT, 0, s>>>(outer, n, a, nj.lv[0], b, nj.lv[1],
                                                           nullptr, off, out, nullptr);
  return hipGetLastError();
}

#define HL_INSTANTIATE(K)                                                                     \
  template hipError_t join_nested<K>(const K*, u64, const NestedJoin<K>&, u32*, u64*, u64*,  \
                                     u32*, void*, K*, hipStream_t);                           \
  template hipError_t join_probe<K>(const K*, u64, const JoinSpec&, const Slot*, u64, u32*,  \
                                    u32*, hipStream_t, LaunchTimer*);                         \
  template hipError_t join_expand_tiles<K>(const K*, u64, const u64*, const u32*, const K*,  \
                                           u64, const JoinSpec&, const u64*, u64, u64, K*,   \
                                           u64*, hipStream_t, LaunchTimer*, int, const K*,   \
                                           u64);                                               \
  template hipError_t join_expand<K>(const K*, u64, const u64*, const u32*, const K*, u64,  \
                                     const JoinSpec&, u64*, K*, u64*, hipStream_t,            \
                                     LaunchTimer*, int, const K*, u64);                        \
  template hipError_t project<K>(const K*, u64, const JoinSpec&, K*, u64*, hipStream_t);   \
  template hipError_t wide_expand_tiles<K>(const K*, u64, const u64*, const u32*, const K*,  \
                                           u64, const WideSpec&, const u64*, u64, u64, K*,   \
                                           u64*, hipStream_t, LaunchTimer*);                  \
  template hipError_t join_probe_learned<K>(const K*, u64, const JoinSpec&,                  \
                                            const LearnedView<K>&, u32*, u32*, hipStream_t,  \
                                            LaunchTimer*);
HL_INSTANTIATE(u32)
HL_INSTANTIATE(u64)
#undef HL_INSTANTIATE

}  // namespace hl
