// Relations of arity up to 4 and join keys of several columns (the paper's
// requirement R3, "Multiple Join Columns", Section 3; the HISA of Section 4
// built on a prefix of several columns; "Implementing Joins" of Section 5.1,
// whose Foo/Bar example joins on two columns).
//
// A tuple of arity a is a packed key of a*w bits with column 0 in the most
// significant position, so sorting the keys sorts the tuples
// lexicographically in declared column order.  An index of a relation is
// the relation with its columns permuted so that the nj join columns come
// first, sorted; a tuple's join key is then the prefix key >> ((a - nj) * w)
// of up to 64 bits.
//
// The hash index maps the prefix to its run: the slot's key word holds a
// 32-bit fingerprint of the prefix (the paper stores a hash of the join
// columns), plus the run's length, and its second word the run's start.  A
// probe that meets its own fingerprint compares the prefix of the tuple at
// the run's start with its own and probes on when they differ, so prefixes
// whose fingerprints collide never share a run.
#include "device.hpp"
#include "kernels.hpp"

namespace hl {

namespace {

constexpr int kNT = 256;
constexpr int kTileItems = 8;
constexpr u64 kTile = u64(kNT) * kTileItems;

template <typename K>
__device__ __forceinline__ K wcol(K k, int c, int a, int w) {
  return (k >> ((a - 1 - c) * w)) & ((K(1) << w) - 1);
}

// 32-bit fingerprint of a prefix (a mix of both halves).
template <typename K>
__device__ __forceinline__ u32 fingerprint(K p) {
  const u64 x = u64(p);
  return mix32(u32(x) ^ mix32(u32(x >> 32) + 0x9e3779b9u));
}

// The probe value of an outer tuple: its columns jo[0..nj) side by side.
template <typename K>
__device__ __forceinline__ K probe_value(K ok, const WideSpec& ws) {
  K p = 0;
  for (int t = 0; t < ws.nj; ++t) p = (p << ws.w) | wcol(ok, ws.jo[t], ws.ao, ws.w);
  return p;
}

template <typename K>
__global__ __launch_bounds__(kNT) void wide_count_runs_kernel(const K* keys, u64 n, int shift,
                                                              u64* d_runs) {
  __shared__ u64 lds[kNT / kWave];
  u64 c = 0;
  for (u64 i = u64(blockIdx.x) * kNT + threadIdx.x; i < n; i += u64(gridDim.x) * kNT)
    c += (i == 0 || K(keys[i] >> shift) != K(keys[i - 1] >> shift)) ? 1 : 0;
  c = block_sum<kNT>(c, lds);
  if (threadIdx.x == 0 && c)
    atomicAdd(reinterpret_cast<unsigned long long*>(d_runs), (unsigned long long)c);
}

// The first tuple of each run inserts (fingerprint, length, start).
template <typename K>
__global__ __launch_bounds__(kNT) void wide_build_kernel(const K* keys, u64 n, int shift,
                                                         Slot* table, u64 cap) {
  const u64 i = u64(blockIdx.x) * kNT + threadIdx.x;
  if (i >= n) return;
  const K p = keys[i] >> shift;
  if (i > 0 && K(keys[i - 1] >> shift) == p) return;
  u64 lo = i, step = 1;
  while (lo + step < n && K(keys[lo + step] >> shift) == p) {
    lo += step;
    step <<= 1;
  }
  u64 hi = (lo + step < n) ? lo + step : n;
  while (hi - lo > 1) {
    const u64 mid = lo + ((hi - lo) >> 1);
    if (K(keys[mid] >> shift) == p) lo = mid;
    else hi = mid;
  }
  const u32 fp = fingerprint(p);
  const u64 word = ((hi - i) << 32) | u64(fp);  // nonzero: a run is never empty
  u64 slot = slot_of(fp, cap);
  for (u64 probe = 0; probe < cap; ++probe) {
    const unsigned long long prev = atomicCAS(
        reinterpret_cast<unsigned long long*>(&table[slot].w0), 0ull, (unsigned long long)word);
    if (prev == 0ull) {
      table[slot].w1 = i;
      return;
    }
    slot = (slot + 1 == cap) ? 0 : slot + 1;
  }
}

template <typename K>
__device__ __forceinline__ bool wide_find(const Slot* table, u64 cap, const K* inner, int shift,
                                          K p, u32& start, u32& len) {
  const u32 fp = fingerprint(p);
  u64 slot = slot_of(fp, cap);
  for (u64 probe = 0; probe < cap; ++probe) {
    const Slot sl = table[slot];
    if (sl.w0 == 0) return false;
    if (u32(sl.w0) == fp && K(inner[sl.w1] >> shift) == p) {
      len = u32(sl.w0 >> 32);
      start = u32(sl.w1);
      return true;
    }
    slot = (slot + 1 == cap) ? 0 : slot + 1;
  }
  return false;
}

// One lane per outer tuple; neighbours with equal probe values share one
// probe (the first lane of each such run in a wave probes).
template <typename K>
__global__ __launch_bounds__(kNT) void wide_probe_kernel(const K* outer, u64 n, WideSpec ws,
                                                         const Slot* table, u64 cap,
                                                         const K* inner, u32* start, u32* len) {
  const u64 i = u64(blockIdx.x) * kNT + threadIdx.x;
  const bool valid = i < n;
  const int shift = (ws.ai - ws.nj) * ws.w;
  K p = 0, prev = 0;
  if (valid) {
    p = probe_value(outer[i], ws);
    if (i > 0) prev = probe_value(outer[i - 1], ws);
  }
  const int lane = lane_id();
  const bool leader = valid && (lane == 0 || i == 0 || p != prev);
  const u64 lm = ballot(leader);
  u32 st = 0, ln = 0;
  if (leader && !wide_find(table, cap, inner, shift, p, st, ln)) ln = 0;
  const u64 upto = lm & ((lane == 63) ? ~u64(0) : ((u64(2) << lane) - 1));
  const int src = upto ? 63 - __clzll((long long)upto) : lane;
  st = __shfl(st, src, kWave);
  ln = __shfl(ln, src, kWave);
  if (valid) {
    start[i] = ln ? st : 0;
    len[i] = ln;
  }
}

// The same through the learned index of the inner array: the run of prefix
// p is [lower_bound(p << shift), lower_bound((p + 1) << shift)).
template <typename K>
__global__ __launch_bounds__(kNT) void wide_probe_learned_kernel(const K* outer, u64 n,
                                                                 WideSpec ws, LearnedView<K> lv,
                                                                 u32* start, u32* len) {
  const u64 i = u64(blockIdx.x) * kNT + threadIdx.x;
  const bool valid = i < n;
  const int shift = (ws.ai - ws.nj) * ws.w;
  const int pbits = ws.nj * ws.w;  // bits of a prefix
  K p = 0, prev = 0;
  if (valid) {
    p = probe_value(outer[i], ws);
    if (i > 0) prev = probe_value(outer[i - 1], ws);
  }
  const int lane = lane_id();
  const bool leader = valid && (lane == 0 || i == 0 || p != prev);
  const u64 lm = ballot(leader);
  u32 st = 0, ln = 0;
  if (leader) {
    st = lm_lower_bound(lv, K(p << shift));
    if (st < lv.n && K(lv.keys[st] >> shift) == p) {
      // the largest prefix has no successor: its run ends the array
      const bool last = pbits >= int(8 * sizeof(K)) ? p == ~K(0)
                                                     : p == (K(1) << pbits) - 1;
      const u32 en = last ? u32(lv.n) : lm_lower_bound(lv, K((p + 1) << shift));
      ln = en - st;
    }
  }
  const u64 upto = lm & ((lane == 63) ? ~u64(0) : ((u64(2) << lane) - 1));
  const int src = upto ? 63 - __clzll((long long)upto) : lane;
  st = __shfl(st, src, kWave);
  ln = __shfl(ln, src, kWave);
  if (valid) {
    start[i] = ln ? st : 0;
    len[i] = ln;
  }
}

// A join with no shared column (a cross product): every outer tuple takes
// the whole inner array.
__global__ __launch_bounds__(kNT) void wide_probe_all_kernel(u64 n, u32 n_inner, u32* start,
                                                             u32* len) {
  const u64 i = u64(blockIdx.x) * kNT + threadIdx.x;
  if (i >= n) return;
  start[i] = 0;
  len[i] = n_inner;
}

// One-atom bodies: each input tuple becomes one head tuple (column sources
// 0..3 of the input, 8 the constant 0), kept if it passes the tests.
template <typename K>
__global__ __launch_bounds__(kNT) void wide_project_kernel(const K* in, u64 n, WideSpec ws,
                                                           K* out, u64* cursor) {
  __shared__ K s_keep[kTile];
  __shared__ u32 s_wsum[kNT / kWave];
  __shared__ u64 s_base;
  __shared__ u32 s_count;
  const bool filtered = ws.nf > 0 || ws.ne > 0;
  const u64 t0 = u64(blockIdx.x) * kTile;
  if (threadIdx.x == 0) s_count = 0;
  __syncthreads();
  for (u32 kk = 0; kk < kTile; kk += kNT) {
    const u64 i = t0 + kk + threadIdx.x;
    bool keep = false;
    K v = 0;
    if (i < n) v = wide_gather(in[i], K(0), ws, keep);
    if (filtered) {
      u32 tot;
      const u32 pos = block_exclusive_scan<kNT>(keep ? 1u : 0u, s_wsum, tot);
      const u32 base = s_count;
      if (keep) s_keep[base + pos] = v;
      __syncthreads();
      if (threadIdx.x == 0) s_count = base + tot;
      __syncthreads();
    } else if (i < n) {
      out[i] = v;
    }
  }
  if (filtered) {
    const u32 c = s_count;
    if (threadIdx.x == 0)
      s_base = c ? atomicAdd(reinterpret_cast<unsigned long long*>(cursor), (unsigned long long)c)
                 : 0;
    __syncthreads();
    for (u32 k = threadIdx.x; k < c; k += kNT) out[s_base + k] = s_keep[k];
  }
}

template <typename K>
__global__ __launch_bounds__(kNT) void wide_permute_kernel(const K* in, u64 n, int a, int w,
                                                           int p0, int p1, int p2, int p3,
                                                           K* out) {
  const int perm[4] = {p0, p1, p2, p3};
  const u64 stride = u64(gridDim.x) * kNT;
  for (u64 i = u64(blockIdx.x) * kNT + threadIdx.x; i < n; i += stride) {
    const K k = in[i];
    K v = 0;
    for (int c = 0; c < a; ++c) v = (v << w) | wcol(k, perm[c], a, w);
    out[i] = v;
  }
}

template <typename K>
__global__ __launch_bounds__(kNT) void wide_pack_kernel(const u32* rows, u64 n, int a, int w,
                                                        K* out) {
  const u64 stride = u64(gridDim.x) * kNT;
  for (u64 i = u64(blockIdx.x) * kNT + threadIdx.x; i < n; i += stride) {
    K v = 0;
    for (int c = 0; c < a; ++c) v = (v << w) | K(rows[i * a + c]);
    out[i] = v;
  }
}

template <typename K>
__global__ __launch_bounds__(kNT) void wide_unpack_kernel(const K* keys, u64 n, int a, int w,
                                                          u32* rows, u32 sub) {
  const u64 stride = u64(gridDim.x) * kNT;
  for (u64 i = u64(blockIdx.x) * kNT + threadIdx.x; i < n; i += stride) {
    const K k = keys[i];
    for (int c = 0; c < a; ++c) rows[i * a + c] = u32(wcol(k, c, a, w)) - sub;
  }
}

u32 grid_for(u64 n, u64 cap_blocks = 65536) {
  u64 b = (n + kNT - 1) / kNT;
  if (b == 0) b = 1;
  return u32(b < cap_blocks ? b : cap_blocks);
}

bool spec_ok(const WideSpec& ws) {
  if (ws.w < 1 || ws.w > 32 || ws.ao < 1 || ws.ao > 4 || ws.ai < 0 || ws.ai > 4) return false;
  if (ws.nj < 0 || ws.nj > ws.ai || ws.nout < 1 || ws.nout > 4) return false;
  if (ws.nf < 0 || ws.nf > 4 || ws.ne < 0 || ws.ne > 4) return false;
  for (int t = 0; t < ws.nj; ++t)
    if (ws.jo[t] < 0 || ws.jo[t] >= ws.ao) return false;
  return true;
}

}  // namespace

bool wide_spec_ok(const WideSpec& ws) { return spec_ok(ws); }

template <typename K>
hipError_t wide_count_runs(const K* keys, u64 n, int shift, u64* d_runs, hipStream_t s) {
  hipError_t e = fill_zero(d_runs, sizeof(u64), s);
  if (e != hipSuccess || n == 0) return e;
  wide_count_runs_kernel<K><<<grid_for(n, 8192), kNT, 0, s>>>(keys, n, shift, d_runs);
  return hipGetLastError();
}

template <typename K>
hipError_t wide_hisa_build(const K* keys, u64 n, int shift, Slot* table, u64 cap, hipStream_t s,
                           LaunchTimer* timer) {
  if (n == 0) return hipSuccess;
  if (cap == 0 || cap > (u64(1) << 32) || n >= (u64(1) << 32)) return hipErrorInvalidValue;
  const u64 blocks = (n + kNT - 1) / kNT;
  if (timer) timer->begin(K_HISA_BUILD, s);
  wide_build_kernel<K><<<dim3(u32(blocks)), kNT, 0, s>>>(keys, n, shift, table, cap);
  if (timer) timer->end(K_HISA_BUILD, s, n * sizeof(K));
  return hipGetLastError();
}

template <typename K>
hipError_t wide_probe(const K* outer, u64 n, const WideSpec& ws, const Slot* table, u64 cap,
                      const K* inner, u32* start, u32* len, hipStream_t s, LaunchTimer* timer) {
  if (n == 0) return hipSuccess;
  if (!spec_ok(ws) || ws.nj < 1 || cap == 0 || cap > (u64(1) << 32)) return hipErrorInvalidValue;
  const u64 blocks = (n + kNT - 1) / kNT;
  if (blocks >= (u64(1) << 31)) return hipErrorInvalidValue;
  if (timer) timer->begin(K_JOIN_PROBE, s);
  wide_probe_kernel<K><<<dim3(u32(blocks)), kNT, 0, s>>>(outer, n, ws, table, cap, inner, start,
                                                         len);
  if (timer) timer->end(K_JOIN_PROBE, s, n * (sizeof(K) + sizeof(Slot) + 2 * sizeof(u32)));
  return hipGetLastError();
}

hipError_t wide_probe_all(u64 n, u64 n_inner, u32* start, u32* len, hipStream_t s,
                          LaunchTimer* timer) {
  if (n == 0) return hipSuccess;
  if (n_inner >= (u64(1) << 32)) return hipErrorInvalidValue;
  const u64 blocks = (n + kNT - 1) / kNT;
  if (blocks >= (u64(1) << 31)) return hipErrorInvalidValue;
  if (timer) timer->begin(K_JOIN_PROBE, s);
  wide_probe_all_kernel<<<dim3(u32(blocks)), kNT, 0, s>>>(n, u32(n_inner), start, len);
  if (timer) timer->end(K_JOIN_PROBE, s, n * 2 * sizeof(u32));
  return hipGetLastError();
}

template <typename K>
hipError_t wide_probe_learned(const K* outer, u64 n, const WideSpec& ws, const LearnedView<K>& lv,
                              u32* start, u32* len, hipStream_t s, LaunchTimer* timer) {
  if (n == 0) return hipSuccess;
  if (!spec_ok(ws) || ws.nj < 1 || lv.n >= (u64(1) << 32)) return hipErrorInvalidValue;
  const u64 blocks = (n + kNT - 1) / kNT;
  if (blocks >= (u64(1) << 31)) return hipErrorInvalidValue;
  if (timer) timer->begin(K_JOIN_PROBE, s);
  wide_probe_learned_kernel<K><<<dim3(u32(blocks)), kNT, 0, s>>>(outer, n, ws, lv, start, len);
  if (timer) timer->end(K_JOIN_PROBE, s, n * (sizeof(K) + 2 * sizeof(u32)));
  return hipGetLastError();
}

template <typename K>
hipError_t wide_project(const K* in, u64 n, const WideSpec& ws, K* out, u64* cursor,
                        hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (!spec_ok(ws)) return hipErrorInvalidValue;
  const u64 blocks = (n + kTile - 1) / kTile;
  if (blocks >= (u64(1) << 31)) return hipErrorInvalidValue;
  wide_project_kernel<K><<<dim3(u32(blocks)), kNT, 0, s>>>(in, n, ws, out, cursor);
  return hipGetLastError();
}

template <typename K>
hipError_t wide_permute(const K* in, u64 n, int a, int w, const int* perm, K* out,
                        hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (a < 1 || a > 4) return hipErrorInvalidValue;
  int p[4] = {0, 1, 2, 3};
  for (int c = 0; c < a; ++c) {
    if (perm[c] < 0 || perm[c] >= a) return hipErrorInvalidValue;
    p[c] = perm[c];
  }
  wide_permute_kernel<K><<<grid_for(n), kNT, 0, s>>>(in, n, a, w, p[0], p[1], p[2], p[3], out);
  return hipGetLastError();
}

template <typename K>
hipError_t wide_pack(const u32* rows, u64 n, int a, int w, K* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (a < 1 || a > 4) return hipErrorInvalidValue;
  wide_pack_kernel<K><<<grid_for(n), kNT, 0, s>>>(rows, n, a, w, out);
  return hipGetLastError();
}

template <typename K>
hipError_t wide_unpack(const K* keys, u64 n, int a, int w, u32* rows, hipStream_t s, u32 sub) {
  if (n == 0) return hipSuccess;
  if (a < 1 || a > 4) return hipErrorInvalidValue;
  wide_unpack_kernel<K><<<grid_for(n), kNT, 0, s>>>(keys, n, a, w, rows, sub);
  return hipGetLastError();
}

#define HL_INSTANTIATE(K)                                                                      \
  template hipError_t wide_count_runs<K>(const K*, u64, int, u64*, hipStream_t);             \
  template hipError_t wide_hisa_build<K>(const K*, u64, int, Slot*, u64, hipStream_t,        \
                                         LaunchTimer*);                                        \
  template hipError_t wide_probe<K>(const K*, u64, const WideSpec&, const Slot*, u64,       \
                                    const K*, u32*, u32*, hipStream_t, LaunchTimer*);          \
  template hipError_t wide_probe_learned<K>(const K*, u64, const WideSpec&,                  \
                                            const LearnedView<K>&, u32*, u32*, hipStream_t,   \
                                            LaunchTimer*);                                     \
  template hipError_t wide_project<K>(const K*, u64, const WideSpec&, K*, u64*, hipStream_t); \
  template hipError_t wide_permute<K>(const K*, u64, int, int, const int*, K*, hipStream_t); \
  template hipError_t wide_pack<K>(const u32*, u64, int, int, K*, hipStream_t);              \
  template hipError_t wide_unpack<K>(const K*, u64, int, int, u32*, hipStream_t, u32);
HL_INSTANTIATE(u32)
HL_INSTANTIATE(u64)
#undef HL_INSTANTIATE

}  // namespace hl
