// One fused launch per small iteration: every rule of the recursive
// stratum, for all its delta variants, runs in a single workgroup that
// joins the deltas with the (EDB) inner indexes (Algorithm 3), sorts and
// deduplicates the new tuples in LDS (Section 4.2, sort + unique), drops
// those already in full (Section 5.1, populating delta) and writes each
// relation's new delta.  A merge whose sizes are read from device memory
// (Section 4.2, merge) follows, so the whole iteration, with one small
// device-to-host copy of the counts at its end, can be captured once in a
// HIP graph and replayed while the deltas stay small.
//
// The merge does not rewrite full: new deltas are merged into a short
// sorted tail run kept beside it (full and tail are disjoint, the relation
// is their union, and membership tests search both).  An iteration then
// moves O(|tail| + |delta|) bytes instead of O(|full|); the engine folds
// the tail into full when the fused iterations end or the tail outgrows
// its buffer.
//
// This is for the tail of long fixpoints, where each delta is a few
// thousand tuples: there the multi-kernel path costs dozens of launches and
// two host synchronisations per iteration for microseconds of work.  The
// kernel holds every candidate in LDS; when an iteration's joins produce
// more than fit, it writes nothing but an overflow flag and the engine runs
// that iteration on the multi-kernel path instead (the inputs are not
// modified, so the rerun starts from the same state).
#include "device.hpp"
#include "kernels.hpp"

namespace hl {

namespace {

constexpr int kFNT = kFusedThreads;  // one workgroup of 1024 threads
constexpr int kFWaves = kFNT / kWave;
constexpr int kLock = 4;  // membership searches in flight per thread
static_assert(kFusedGroups < kFNT, "one finishing thread per phase-A workgroup");

// Value number src of (c0, c1, inner's other column); 3 is the constant 0.
template <typename K>
__device__ __forceinline__ K fz_pick(int src, K c0, K c1, K o) {
  return src == 0 ? c0 : (src == 1 ? c1 : (src == 2 ? o : K(0)));
}

__device__ __forceinline__ bool fz_hash_find(const Slot* table, u64 cap, u32 key, u32& start,
                                             u32& len) {
  u64 slot = slot_of(key, cap);
  for (u64 probe = 0; probe < cap; ++probe) {
    const Slot sl = table[slot];
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

// Run [start, start + len) of join key jc in the inner sorted array.
template <typename K>
__device__ __forceinline__ void fz_probe(const FusedStep<K>& s, u32 jc, int w, u32& start,
                                         u32& len) {
  start = 0;
  len = 0;
  if (s.table) {
    if (!fz_hash_find(s.table, s.cap, jc, start, len)) len = 0;
    return;
  }
  const LearnedView<K>& lv = s.lv;
  const u32 st = lm_lower_bound(lv, K(jc) << w);
  if (st >= lv.n || K(lv.keys[st] >> w) != K(jc)) return;
  // the next key's first position; when jc is the largest id, the shifted
  // key wraps to 0 and the run ends with the array
  const K next = (K(jc) + 1) << w;
  const u32 en = next == 0 ? u32(lv.n) : lm_lower_bound(lv, next);
  start = st;
  len = en - st;
}

// Appends the kept values of one round (at most one per thread) to dst at
// *count, in thread order.  Returns false (for every thread) when they do
// not fit in cap.  Every thread must call it.
template <typename K>
__device__ __forceinline__ bool fz_append(K v, bool keep, K* dst, u32& count, u32 cap,
                                          u32* wsum) {
  u32 tot;
  const u32 pos = block_exclusive_scan<kFNT>(keep ? 1u : 0u, wsum, tot);
  if (count + tot > cap) return false;
  if (keep) dst[count + pos] = v;
  count += tot;
  return true;
}

// Ascending bitonic sort of a[0, p) in LDS, p a power of two; every thread
// must call it.
template <typename K>
__device__ void fz_bitonic(K* a, u32 p) {
  for (u32 k = 2; k <= p; k <<= 1) {
    for (u32 j = k >> 1; j > 0; j >>= 1) {
      for (u32 i = threadIdx.x; i < p / 2; i += kFNT) {
        const u32 lo = 2 * j * (i / j) + (i % j), hi = lo + j;
        const bool up = (lo & k) == 0;
        const K x = a[lo], y = a[hi];
        if ((x > y) == up) {
          a[lo] = y;
          a[hi] = x;
        }
      }
      __syncthreads();
    }
  }
}

// keep[r] &= (key[r] is not in the sorted array a[0, n)), for the kLock
// keys of this thread, searched in lockstep.
template <typename K>
__device__ __forceinline__ void fz_drop_members(const K* a, u64 n, const K* key, bool* keep) {
  if (n == 0) return;
  int steps = 0;
  while ((u64(1) << steps) <= n) ++steps;
  u64 lo[kLock], hi[kLock];
#pragma unroll
  for (int r = 0; r < kLock; ++r) {
    lo[r] = 0;
    hi[r] = keep[r] ? n : 0;
  }
  for (int t = 0; t < steps; ++t) {
#pragma unroll
    for (int r = 0; r < kLock; ++r) {
      if (lo[r] < hi[r]) {
        const u64 mid = (lo[r] + hi[r]) >> 1;
        if (a[mid] < key[r]) lo[r] = mid + 1;
        else hi[r] = mid;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kLock; ++r)
    if (keep[r] && lo[r] < n && a[lo[r]] == key[r]) keep[r] = false;
}

// The same through a learned index over a: each key's search starts from
// the model's window, which holds its lower bound exactly.
template <typename K>
__device__ __forceinline__ void fz_drop_members_lm(const LearnedView<K>& lv, const K* key,
                                                   bool* keep) {
  u64 lo[kLock], hi[kLock];
#pragma unroll
  for (int r = 0; r < kLock; ++r) {
    lo[r] = hi[r] = 0;
    if (keep[r]) lm_window(lv, key[r], lo[r], hi[r]);
  }
  bool busy = true;
  while (busy) {
    busy = false;
#pragma unroll
    for (int r = 0; r < kLock; ++r) {
      if (lo[r] < hi[r]) {
        const u64 mid = (lo[r] + hi[r]) >> 1;
        if (lv.keys[mid] < key[r]) lo[r] = mid + 1;
        else hi[r] = mid;
        busy = true;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kLock; ++r)
    if (keep[r] && lo[r] < lv.n && lv.keys[lo[r]] == key[r]) keep[r] = false;
}

// Phase A: workgroup g of G takes the g-th slice of every delta, joins it,
// sorts and deduplicates its candidates in LDS, and tests each distinct one
// against full and the tail.  It writes two sorted runs per head: the
// candidates that are new (survivors) and those already present, and its
// counts.  Duplicates across workgroups remain; phase B removes them.
template <typename K>
__global__ __launch_bounds__(kFNT) void fused_join_kernel(FusedIteration<K> it, u32 cap_c,
                                                          u32 cap_t, FusedScratch<K> sc) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  K* cand = reinterpret_cast<K*>(s_dyn);     // cap_c keys: one head's new tuples
  K* tmpb = cand + cap_c;                    // cap_t keys: a first join's result
  K* s_outer = tmpb + cap_t;                 // kFNT: the chunk's outer tuples
  u32* s_off = reinterpret_cast<u32*>(s_outer + kFNT);  // kFNT: their output offsets
  u32* s_start = s_off + kFNT;               // kFNT: their run starts
  __shared__ u32 s_wsum[kFWaves];
  u64* cnt = it.counts;
  const int w = it.w;
  const K mask = (K(1) << w) - 1;
  const u32 G = gridDim.x, g = blockIdx.x;

  for (int h = 0; h < it.nrels; ++h) {
    u32 m = 0;       // candidates of head h in cand
    u64 raw = 0;     // join outputs of head h before filters
    for (int pi = 0; pi < it.nplans; ++pi) {
      const FusedPlan<K>& p = it.plans[pi];
      if (p.head != h) continue;
      const u64 n_all = cnt[p.outer * kFusedSlots + 0];
      const u64 lo_i = n_all * g / G, hi_i = n_all * (g + 1) / G;
      const K* cur = it.delta_in[p.outer] + lo_i;
      u32 n = u32(hi_i - lo_i);
      if (p.nsteps == 0) {
        const JoinSpec& js = p.steps[0].js;
        for (u32 b = 0; b < n; b += kFNT) {
          const u32 i = b + threadIdx.x;
          K v = 0;
          bool keep = false;
          if (i < n) {
            const K k = cur[i];
            const K c0 = k >> w, c1 = k & mask;
            v = (fz_pick(js.src0, c0, c1, K(0)) << w) | fz_pick(js.src1, c0, c1, K(0));
            keep = (js.fa < 0 || fz_pick(js.fa, c0, c1, K(0)) != fz_pick(js.fb, c0, c1, K(0))) &&
                   (js.ea < 0 || fz_pick(js.ea, c0, c1, K(0)) == fz_pick(js.eb, c0, c1, K(0)));
          }
          raw += (n - b < u32(kFNT)) ? n - b : u32(kFNT);
          if (!fz_append(v, keep, cand, m, cap_c, s_wsum)) goto overflow;
        }
        continue;
      }
      for (int q = 0; q < p.nsteps; ++q) {
        const FusedStep<K>& s = p.steps[q];
        const JoinSpec& js = s.js;
        const bool last = q + 1 == p.nsteps;
        K* dst = last ? cand : tmpb;
        u32 dcount = last ? m : 0;
        const u32 dcap = last ? cap_c : cap_t;
        for (u32 b = 0; b < n; b += kFNT) {
          // one outer tuple per thread: its run in the inner index
          const u32 i = b + threadIdx.x;
          K ok = 0;
          u32 st = 0, ln = 0;
          if (i < n) {
            ok = cur[i];
            const u32 jc = js.outer_col == 0 ? u32(ok >> w) : u32(ok & mask);
            fz_probe(s, jc, w, st, ln);
          }
          // more outputs than the destination holds is an overflow even if
          // filters would drop some (clamping keeps the sum within 32 bits)
          u32 total;
          const u32 off = block_exclusive_scan<kFNT>(ln < dcap ? ln : dcap + 1, s_wsum, total);
          if (dcount + u64(total) > dcap) goto overflow;
          s_outer[threadIdx.x] = ok;
          s_off[threadIdx.x] = off;
          s_start[threadIdx.x] = st;
          __syncthreads();
          if (last) raw += total;
          for (u32 ob = 0; ob < total; ob += kFNT) {
            const u32 o = ob + threadIdx.x;
            K v = 0;
            bool keep = false;
            if (o < total) {
              // owner: the last outer tuple whose offset is <= o (it has a
              // nonempty run, since the next offset is > o)
              u32 lo = 0, hi = kFNT;
              while (hi - lo > 1) {
                const u32 mid = (lo + hi) >> 1;
                if (s_off[mid] <= o) lo = mid;
                else hi = mid;
              }
              const K k = s_outer[lo];
              const K c0 = k >> w, c1 = k & mask;
              const K oth = s.inner[u64(s_start[lo]) + (o - s_off[lo])] & mask;
              v = (fz_pick(js.src0, c0, c1, oth) << w) | fz_pick(js.src1, c0, c1, oth);
              keep = (js.fa < 0 || fz_pick(js.fa, c0, c1, oth) != fz_pick(js.fb, c0, c1, oth)) &&
                     (js.ea < 0 || fz_pick(js.ea, c0, c1, oth) == fz_pick(js.eb, c0, c1, oth));
            }
            if (!fz_append(v, keep, dst, dcount, dcap, s_wsum)) goto overflow;
          }
          __syncthreads();  // s_outer / s_off / s_start are rewritten next chunk
        }
        if (last) {
          m = dcount;
        } else {
          cur = tmpb;
          n = dcount;
          __syncthreads();
        }
      }
    }
    {
      // sort: pad to a power of two with the largest key (a pad equal to a
      // real key is indistinguishable from it, so the first m stay right)
      u32 p2 = 2;
      while (p2 < m) p2 <<= 1;
      for (u32 k = m + threadIdx.x; k < p2; k += kFNT) cand[k] = ~K(0);
      __syncthreads();
      if (m > 1) fz_bitonic(cand, p2);
      // unique, then split by membership in full or the tail: kLock binary
      // searches per thread advance in lockstep so their dependent loads
      // overlap
      const K* full = it.full[h];
      const u64 nf = cnt[h * kFusedSlots + 1];
      const K* tail = it.tail[h];
      const u64 ntl = cnt[h * kFusedSlots + 6];
      const u64 slot = u64(h) * G + g;
      K* surv = sc.surv + slot * cap_c;
      K* pres = sc.pres + slot * cap_c;
      u32 ns = 0, np = 0;
      for (u32 b = 0; b < m; b += kFNT * kLock) {
        K key[kLock];
        bool first[kLock], keep[kLock];
#pragma unroll
        for (int r = 0; r < kLock; ++r) {
          const u32 i = b + u32(r) * kFNT + threadIdx.x;
          first[r] = i < m && (i == 0 || cand[i - 1] != cand[i]);
          key[r] = i < m ? cand[i] : K(0);
          keep[r] = first[r];
        }
        if (it.full_lm[h].n == nf && nf > 0 && it.full_lm[h].keys == full)
          fz_drop_members_lm(it.full_lm[h], key, keep);
        else
          fz_drop_members(full, nf, key, keep);
        fz_drop_members(tail, ntl, key, keep);
#pragma unroll
        for (int r = 0; r < kLock; ++r) {
          u32 tot;
          u32 pos = block_exclusive_scan<kFNT>(keep[r] ? 1u : 0u, s_wsum, tot);
          if (keep[r]) surv[ns + pos] = key[r];
          ns += tot;
          const bool old = first[r] && !keep[r];
          pos = block_exclusive_scan<kFNT>(old ? 1u : 0u, s_wsum, tot);
          if (old) pres[np + pos] = key[r];
          np += tot;
        }
      }
      if (threadIdx.x == 0) {
        u64* c = sc.counts + slot * 4;
        c[0] = ns;
        c[1] = np;
        c[2] = m;
        c[3] = raw;
      }
      __syncthreads();
    }
  }
  return;
overflow:
  if (threadIdx.x == 0) cnt[kFusedOverflow] = 1;
}

// Copies the sorted runs of head h from every phase-A workgroup into
// dst[0, total): `off` holds the G + 1 run offsets (exclusive prefix of the
// run lengths, in LDS).  Each output position finds its run by a binary
// search of the offsets, so all runs are copied at once.
template <typename K>
__device__ void fz_gather(const K* runs, int h, u32 G, u32 cap, const u32* off, K* dst) {
  const u32 total = off[G];
  for (u32 k = threadIdx.x; k < total; k += kFNT) {
    u32 lo = 0, hi = G;  // off[lo] <= k < off[hi]
    while (hi - lo > 1) {
      const u32 mid = (lo + hi) >> 1;
      if (off[mid] <= k) lo = mid;
      else hi = mid;
    }
    dst[k] = runs[(u64(h) * G + lo) * cap + (k - off[lo])];
  }
  __syncthreads();
}

// Exclusive prefix of the phase-A run lengths of head h (`which`: 0
// survivors, 1 present) into off[0, G]; every thread must call it.
__device__ __forceinline__ u32 fz_offsets(const u64* counts, int h, u32 G, int which, u32* off,
                                          u32* wsum) {
  const u32 g = threadIdx.x;
  const u32 n = g < G ? u32(counts[(u64(h) * G + g) * 4 + which]) : 0u;
  u32 total;
  const u32 x = block_exclusive_scan<kFNT>(n, wsum, total);
  if (g <= G) off[g] = x;
  __syncthreads();
  return total;
}

// Sorts buf[0, n), the concatenation of R sorted runs with offsets
// ro[0, R] (LDS; rewritten), and returns where the sorted keys are.  With
// n <= cap / 2 the runs are merged pairwise, ping-ponging with the upper
// half of the buffer: each thread takes 8 consecutive outputs, finds its
// pair of runs (the first whose end is past its first output), splits the
// pair by a merge-path search and merges serially (ties: the earlier run
// first).  log2(R) rounds cost far fewer LDS accesses than a bitonic
// network over the same keys.  Larger inputs take the bitonic sort.
// Every thread must call it.
template <typename K>
__device__ K* fz_sort_runs(K* buf, u32 n, u32 cap, u32* ro, u32 R) {
  if (n <= 1) return buf;
  if (n > cap / 2) {
    u32 p2 = 2;
    while (p2 < n) p2 <<= 1;
    for (u32 k = n + threadIdx.x; k < p2; k += kFNT) buf[k] = ~K(0);
    __syncthreads();
    fz_bitonic(buf, p2);
    return buf;
  }
  constexpr u32 kSpan = 8;
  K* src = buf;
  K* dst = buf + cap / 2;
  while (R > 1) {
    const u32 R2 = (R + 1) / 2;
    for (u32 c0 = threadIdx.x * kSpan; c0 < n; c0 += kFNT * kSpan) {
      const u32 c1 = (c0 + kSpan) < n ? (c0 + kSpan) : n;
      u32 k = c0;
      while (k < c1) {
        // pair i covers runs 2i and 2i + 1: [ro[2i], ro[min(2i + 2, R)])
        u32 lo = 0, hi = R2 - 1;
        while (lo < hi) {
          const u32 mid = (lo + hi) >> 1;
          const u32 e = 2 * mid + 2 < R ? 2 * mid + 2 : R;
          if (ro[e] > k) hi = mid;
          else lo = mid + 1;
        }
        const u32 a0 = ro[2 * lo];
        const u32 a1 = ro[2 * lo + 1 < R ? 2 * lo + 1 : R];
        const u32 b1 = ro[2 * lo + 2 < R ? 2 * lo + 2 : R];
        if (b1 <= k) break;  // cannot happen (ro[R] == n > k); never loops
        const u32 la = a1 - a0, lb = b1 - a1, diag = k - a0;
        u32 alo = diag > lb ? diag - lb : 0, ahi = diag < la ? diag : la;
        while (alo < ahi) {
          const u32 mid = (alo + ahi) >> 1;
          if (!(src[a1 + (diag - 1 - mid)] < src[a0 + mid])) alo = mid + 1;
          else ahi = mid;
        }
        u32 ai = alo, bi = diag - alo;
        const u32 end = c1 < b1 ? c1 : b1;
        for (; k < end; ++k) {
          const bool take_a = bi >= lb || (ai < la && !(src[a1 + bi] < src[a0 + ai]));
          dst[k] = take_a ? src[a0 + ai++] : src[a1 + bi++];
        }
      }
    }
    __syncthreads();
    // the merged runs start where the even runs started
    const u32 j = threadIdx.x;
    u32 v = 0;
    if (j < R2) v = ro[2 * j];
    __syncthreads();
    if (j < R2) ro[j] = v;
    if (j == R2) ro[j] = n;
    __syncthreads();
    R = R2;
    K* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// Number of distinct keys in the sorted a[0, n); every thread must call it.
template <typename K>
__device__ u32 fz_count_distinct(const K* a, u32 n, u32* wsum) {
  u32 d = 0;
  for (u32 b = 0; b < n; b += kFNT) {
    const u32 i = b + threadIdx.x;
    const bool first = i < n && (i == 0 || a[i - 1] != a[i]);
    d += block_sum<kFNT>(first ? 1u : 0u, wsum);
  }
  return d;
}

// Phase B, one workgroup: the survivors of all workgroups are sorted and
// deduplicated into each head's new delta; the distinct count adds the
// distinct present candidates.  After an overflow in either phase no
// relation gets a delta.
template <typename K>
__global__ __launch_bounds__(kFNT) void fused_finish_kernel(FusedIteration<K> it, u32 cap_c,
                                                            u32 cap_b, u32 G, FusedScratch<K> sc) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  K* buf = reinterpret_cast<K*>(s_dyn);  // cap_b keys (runs are cap_c apart)
  __shared__ u32 s_wsum[kFWaves];
  __shared__ u32 s_off[kFusedGroups + 1];
  __shared__ u64 s_sum[2][kFWaves];
  u64* cnt = it.counts;
  if (cnt[kFusedOverflow] != 0) goto overflow;
  for (int h = 0; h < it.nrels; ++h) {
    // candidates and join outputs: sums over the workgroups
    u64 m = 0, raw = 0;
    {
      const u32 g = threadIdx.x;
      const u64 mg = g < G ? sc.counts[(u64(h) * G + g) * 4 + 2] : 0;
      const u64 rg = g < G ? sc.counts[(u64(h) * G + g) * 4 + 3] : 0;
      m = block_sum<kFNT>(mg, s_sum[0]);
      raw = block_sum<kFNT>(rg, s_sum[1]);
    }
    u32 n = fz_offsets(sc.counts, h, G, 0, s_off, s_wsum);
    if (n > cap_b) goto overflow;
    fz_gather(sc.surv, h, G, cap_c, s_off, buf);
    const K* srt = fz_sort_runs(buf, n, cap_b, s_off, G);
    K* out = it.delta_out[h];
    u32 d = 0;
    for (u32 b = 0; b < n; b += kFNT) {
      const u32 i = b + threadIdx.x;
      const bool first = i < n && (i == 0 || srt[i - 1] != srt[i]);
      u32 tot;
      const u32 pos = block_exclusive_scan<kFNT>(first ? 1u : 0u, s_wsum, tot);
      if (first) out[d + pos] = srt[i];
      d += tot;
    }
    __syncthreads();
    n = fz_offsets(sc.counts, h, G, 1, s_off, s_wsum);
    if (n > cap_b) goto overflow;
    fz_gather(sc.pres, h, G, cap_c, s_off, buf);
    srt = fz_sort_runs(buf, n, cap_b, s_off, G);
    const u32 dp = fz_count_distinct(srt, n, s_wsum);
    if (threadIdx.x == 0) {
      cnt[h * kFusedSlots + 2] = d;
      cnt[h * kFusedSlots + 3] = u64(d) + dp;
      cnt[h * kFusedSlots + 4] = m;
      cnt[h * kFusedSlots + 5] = raw;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) cnt[kFusedOverflow] = 0;
  return;
overflow:
  // nothing of this iteration counts: no relation gets a delta
  if (threadIdx.x == 0) {
    for (int r = 0; r < it.nrels; ++r) cnt[r * kFusedSlots + 2] = 0;
    cnt[kFusedOverflow] = 1;
  }
}

// tail' = merge(tail, delta) with both sizes read from the counts; a grid
// larger than needed is fine (surplus tiles return at once).  Nothing runs
// after an overflow or when the delta is empty.
constexpr int kFMNT = 256;
constexpr int kFMItems = 8;
constexpr u64 kFMTile = u64(kFMNT) * kFMItems;

template <typename K>
__device__ __forceinline__ u64 fz_merge_path(const K* a, u64 na, const K* b, u64 nb, u64 diag) {
  u64 lo = diag > nb ? diag - nb : 0;
  u64 hi = diag < na ? diag : na;
  while (lo < hi) {
    const u64 mid = (lo + hi) >> 1;
    if (!(b[diag - 1 - mid] < a[mid])) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <typename K>
__global__ void fz_merge_partition_kernel(const K* a, const K* b, const u64* cnt, int r,
                                          u64* parts, u64 nparts) {
  if (cnt[kFusedOverflow] != 0) return;
  const u64 na = cnt[r * kFusedSlots + 6], nb = cnt[r * kFusedSlots + 2];
  if (nb == 0) return;
  const u64 t = u64(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nparts) return;
  u64 diag = t * kFMTile;
  if (diag > na + nb) diag = na + nb;
  parts[t] = fz_merge_path(a, na, b, nb, diag);
}

template <typename K>
__global__ __launch_bounds__(kFMNT) void fz_merge_kernel(const K* a, const K* b, const u64* cnt,
                                                         int r, const u64* parts, K* out) {
  if (cnt[kFusedOverflow] != 0) return;
  const u64 na = cnt[r * kFusedSlots + 6], nb = cnt[r * kFusedSlots + 2];
  if (nb == 0) return;
  const u64 n = na + nb;
  const u64 tile = blockIdx.x;
  const u64 d0 = tile * kFMTile;
  if (d0 >= n) return;
  // written back padded by one slot per kFMItems keys (distinct banks)
  __shared__ K s[kFMTile + kFMTile / kFMItems];
  const u64 d1 = (d0 + kFMTile) < n ? (d0 + kFMTile) : n;
  const u64 a0 = parts[tile], a1 = parts[tile + 1];
  const u64 b0 = d0 - a0, b1 = d1 - a1;
  const u32 la = u32(a1 - a0), lb = u32(b1 - b0);
  const u32 total = la + lb;
  {
    // both slices side by side, every load issued before any is stored
    K v[kFMItems];
#pragma unroll
    for (int q = 0; q < kFMItems; ++q) {
      const u32 k = u32(q) * kFMNT + threadIdx.x;
      v[q] = k < la ? a[a0 + k] : (k < total ? b[b0 + (k - la)] : K(0));
    }
#pragma unroll
    for (int q = 0; q < kFMItems; ++q) {
      const u32 k = u32(q) * kFMNT + threadIdx.x;
      if (k < total) s[k] = v[q];
    }
  }
  __syncthreads();
  u32 diag = threadIdx.x * kFMItems;
  if (diag > total) diag = total;
  u32 ai = u32(fz_merge_path(s, la, s + la, lb, diag));
  u32 bi = diag - ai;
  K v[kFMItems];
#pragma unroll
  for (int k = 0; k < kFMItems; ++k) {
    K x = 0;
    if (diag + k < total) {
      const bool take_a = (bi >= lb) || (ai < la && !(s[la + bi] < s[ai]));
      if (take_a) x = s[ai++];
      else x = s[la + bi++];
    }
    v[k] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kFMItems; ++k) {
    const u32 o = threadIdx.x * kFMItems + k;
    if (o < total) s[o + o / kFMItems] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kFMItems; ++q) {
    const u32 k = u32(q) * kFMNT + threadIdx.x;
    if (k < total) out[d0 + k] = s[k + k / kFMItems];
  }
}

// After the merges: the new delta is the next iteration's outer and the
// tail has grown by it (only when the iteration did not overflow).
__global__ void fz_advance_kernel(u64* cnt, int nrels) {
  if (threadIdx.x != 0 || cnt[kFusedOverflow] != 0) return;
  for (int r = 0; r < nrels; ++r) {
    const u64 d = cnt[r * kFusedSlots + 2];
    cnt[r * kFusedSlots + 6] += d;
    cnt[r * kFusedSlots + 0] = d;
  }
}

}  // namespace

template <typename K>
u64 fused_lds_bytes(u32 cap_c, u32 cap_t) {
  return u64(cap_c + cap_t + kFNT) * sizeof(K) + 2 * u64(kFNT) * sizeof(u32);
}

template <typename K>
u64 fused_scratch_bytes(u32 cap_c, int nrels) {
  const u64 runs = u64(nrels) * kFusedGroups * cap_c * sizeof(K);
  return 2 * align_up(runs, 256) + align_up(u64(nrels) * kFusedGroups * 4 * sizeof(u64), 256);
}

template <typename K>
hipError_t fused_prepare(u32 cap_c, u32 cap_t, u32 cap_b) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fused_join_kernel<K>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     int(fused_lds_bytes<K>(cap_c, cap_t)));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&fused_finish_kernel<K>),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(u64(cap_b) * sizeof(K)));
}

u64 fused_merge_tiles(u64 n) { return (n + kFMTile - 1) / kFMTile; }

template <typename K>
hipError_t fused_iteration(const FusedIteration<K>& it, u32 cap_c, u32 cap_t, u32 cap_b,
                           void* scratch, hipStream_t s) {
  if (it.nrels < 1 || it.nrels > kFusedMaxRels || it.nplans < 0 || it.nplans > kFusedMaxPlans ||
      cap_c < 2 || (cap_c & (cap_c - 1)) != 0 || cap_b < 2 || (cap_b & (cap_b - 1)) != 0 ||
      !it.counts || !scratch)
    return hipErrorInvalidValue;
  for (int p = 0; p < it.nplans; ++p) {
    const FusedPlan<K>& pl = it.plans[p];
    if (pl.nsteps < 0 || pl.nsteps > kFusedMaxSteps || pl.outer < 0 || pl.outer >= it.nrels ||
        pl.head < 0 || pl.head >= it.nrels)
      return hipErrorInvalidValue;
    for (int q = 0; q < pl.nsteps; ++q)
      if (!pl.steps[q].inner || (!pl.steps[q].table && !pl.steps[q].lv.keys)) return hipErrorInvalidValue;
  }
  FusedScratch<K> sc;
  char* p = static_cast<char*>(scratch);
  const u64 runs = align_up(u64(it.nrels) * kFusedGroups * cap_c * sizeof(K), 256);
  sc.surv = reinterpret_cast<K*>(p);
  sc.pres = reinterpret_cast<K*>(p + runs);
  sc.counts = reinterpret_cast<u64*>(p + 2 * runs);
  fused_join_kernel<K><<<kFusedGroups, kFNT, fused_lds_bytes<K>(cap_c, cap_t), s>>>(it, cap_c,
                                                                                   cap_t, sc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  fused_finish_kernel<K><<<1, kFNT, u64(cap_b) * sizeof(K), s>>>(it, cap_c, cap_b, kFusedGroups,
                                                                   sc);
  return hipGetLastError();
}

template <typename K>
hipError_t fused_merge(const K* tail, const K* delta, const u64* counts, int r, u64 max_out,
                       u64* parts, K* out, hipStream_t s) {
  const u64 nt = fused_merge_tiles(max_out);
  if (nt == 0) return hipSuccess;
  if (nt >= (u64(1) << 31)) return hipErrorInvalidValue;
  const u64 nparts = nt + 1;
  fz_merge_partition_kernel<K><<<dim3(u32((nparts + 255) / 256)), 256, 0, s>>>(tail, delta, counts,
                                                                              r, parts, nparts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  fz_merge_kernel<K><<<dim3(u32(nt)), kFMNT, 0, s>>>(tail, delta, counts, r, parts, out);
  return hipGetLastError();
}

hipError_t fused_advance(u64* counts, int nrels, hipStream_t s) {
  fz_advance_kernel<<<1, 64, 0, s>>>(counts, nrels);
  return hipGetLastError();
}

#define HL_INSTANTIATE(K)                                                                      \
  template u64 fused_lds_bytes<K>(u32, u32);                                                   \
  template u64 fused_scratch_bytes<K>(u32, int);                                               \
  template hipError_t fused_prepare<K>(u32, u32, u32);                                         \
  template hipError_t fused_iteration<K>(const FusedIteration<K>&, u32, u32, u32, void*,       \
                                         hipStream_t);                                         \
  template hipError_t fused_merge<K>(const K*, const K*, const u64*, int, u64, u64*, K*,       \
                                     hipStream_t);
HL_INSTANTIATE(u32)
HL_INSTANTIATE(u64)
#undef HL_INSTANTIATE

}  // namespace hl
