// HISA: hash-indexed sorted array (Section 4).
//
// The sorted array holds packed keys (join column << w) | other column,
// sorted ascending (Section 4.2).  The open-addressing hash index with
// linear probing (Section 4.3) maps a join-column value to the first
// position of its run and, here, also to the run's length, so a range query
// is one 16-byte slot read followed by a contiguous scan.
//
// Build (Algorithm 2 restated): after the sort every run of equal join key
// is contiguous, so exactly one thread (the one at the run's first
// position) inserts each key, claiming an empty slot with a 64-bit CAS.
// The minimum-position race Algorithm 2 resolves with a second CAS loop
// cannot occur.  The slot stores the join key itself rather than its hash
// (it fits in 32 bits), so two keys with equal hashes never share a slot.
//
// Also here: packing of uint32 rows into keys and back, column swap, and
// the max-id reduction that fixes the key width.
#include "device.hpp"
#include "kernels.hpp"

namespace hl {

namespace {

constexpr int kNT = 256;

template <typename K>
__device__ __forceinline__ u32 jkey(K k, int shift) {
  return u32(k >> shift);
}

template <typename K>
__global__ __launch_bounds__(kNT) void count_runs_kernel(const K* keys, u64 n, int shift,
                                                         u64* d_runs) {
  __shared__ u64 lds[kNT / kWave];
  u64 c = 0;
  for (u64 i = u64(blockIdx.x) * kNT + threadIdx.x; i < n; i += u64(gridDim.x) * kNT)
    c += (i == 0 || jkey(keys[i], shift) != jkey(keys[i - 1], shift)) ? 1 : 0;
  c = block_sum<kNT>(c, lds);
  if (threadIdx.x == 0 && c) atomicAdd(reinterpret_cast<unsigned long long*>(d_runs),
                                       (unsigned long long)c);
}

template <typename K>
__global__ __launch_bounds__(kNT) void build_kernel(const K* keys, u64 n, int shift, Slot* table,
                                                    u64 cap) {
  const u64 i = u64(blockIdx.x) * kNT + threadIdx.x;
  if (i >= n) return;
  const u32 jc = jkey(keys[i], shift);
  if (i > 0 && jkey(keys[i - 1], shift) == jc) return;
  // end of the run: gallop, then binary search
  u64 lo = i, step = 1;
  while (lo + step < n && jkey(keys[lo + step], shift) == jc) {
    lo += step;
    step <<= 1;
  }
  u64 hi = (lo + step < n) ? lo + step : n;  // keys[lo] in the run; hi is past it
  while (hi - lo > 1) {
    u64 mid = lo + ((hi - lo) >> 1);
    if (jkey(keys[mid], shift) == jc) lo = mid;
    else hi = mid;
  }
  const u64 len = hi - i;
  const u64 word = (len << 32) | u64(jc);
  u64 slot = slot_of(jc, cap);
  for (u64 probe = 0; probe < cap; ++probe) {
    unsigned long long prev =
        atomicCAS(reinterpret_cast<unsigned long long*>(&table[slot].w0), 0ull,
                  (unsigned long long)word);
    if (prev == 0ull) {
      table[slot].w1 = i;
      return;
    }
    slot = (slot + 1 == cap) ? 0 : slot + 1;
  }
}

__global__ __launch_bounds__(kNT) void probe_kernel(const Slot* table, u64 cap, const u32* q,
                                                    u64 nq, u64* start, u32* len) {
  const u64 i = u64(blockIdx.x) * kNT + threadIdx.x;
  if (i >= nq) return;
  const u32 key = q[i];
  u64 slot = slot_of(key, cap);
  u64 st = 0;
  u32 ln = 0;
  for (u64 probe = 0; probe < cap; ++probe) {
    const Slot sl = table[slot];
    if (sl.w0 == 0) break;
    if (u32(sl.w0) == key) {
      ln = u32(sl.w0 >> 32);
      st = sl.w1;
      break;
    }
    slot = (slot + 1 == cap) ? 0 : slot + 1;
  }
  start[i] = st;
  len[i] = ln;
}

__global__ __launch_bounds__(kNT) void zero_kernel(uint4* p, u64 n16, unsigned char* tail,
                                                   u64 ntail) {
  const u64 stride = u64(gridDim.x) * kNT;
  for (u64 i = u64(blockIdx.x) * kNT + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0)
    for (u64 i = threadIdx.x; i < ntail; i += kNT) tail[i] = 0;
}

__global__ __launch_bounds__(kNT) void max_kernel(const u32* v, u64 n, u32* d_max) {
  u32 m = 0;
  for (u64 i = u64(blockIdx.x) * kNT + threadIdx.x; i < n; i += u64(gridDim.x) * kNT)
    m = v[i] > m ? v[i] : m;
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    u32 o = __shfl_xor(m, d, kWave);
    m = o > m ? o : m;
  }
  if (lane_id() == 0) atomicMax(d_max, m);
}

template <typename K>
__global__ __launch_bounds__(kNT) void pack_kernel(const u32* rows, u64 n, int arity, int w,
                                                   K* out) {
  const u64 stride = u64(gridDim.x) * kNT;
  for (u64 i = u64(blockIdx.x) * kNT + threadIdx.x; i < n; i += stride) {
    K c0 = rows[i * arity];
    K c1 = arity > 1 ? K(rows[i * arity + 1]) : K(0);
    out[i] = (c0 << w) | c1;
  }
}

template <typename K>
__global__ __launch_bounds__(kNT) void swap_kernel(const K* in, u64 n, int w, K* out) {
  const K mask = (K(1) << w) - 1;
  const u64 stride = u64(gridDim.x) * kNT;
  for (u64 i = u64(blockIdx.x) * kNT + threadIdx.x; i < n; i += stride) {
    K k = in[i];
    out[i] = ((k & mask) << w) | (k >> w);
  }
}

template <typename K>
__global__ __launch_bounds__(kNT) void unpack_kernel(const K* keys, u64 n, int arity, int w,
                                                     u32* rows, u32 sub) {
  const K mask = (K(1) << w) - 1;
  const u64 stride = u64(gridDim.x) * kNT;
  for (u64 i = u64(blockIdx.x) * kNT + threadIdx.x; i < n; i += stride) {
    K k = keys[i];
    rows[i * arity] = u32(k >> w) - sub;
    if (arity > 1) rows[i * arity + 1] = u32(k & mask) - sub;
  }
}

template <typename K>
__global__ void key_range_kernel(const K* keys, u64 n, K lo, K hi, u64* out) {
  const int which = threadIdx.x;
  if (which > 1) return;
  const K x = which == 0 ? lo : hi;
  u64 a = 0, b = n;
  while (a < b) {
    u64 mid = (a + b) >> 1;
    if (keys[mid] < x) a = mid + 1;
    else b = mid;
  }
  out[which] = a;
}

u32 grid_for(u64 n, u64 cap_blocks = 65536) {
  u64 b = (n + kNT - 1) / kNT;
  if (b == 0) b = 1;
  return u32(b < cap_blocks ? b : cap_blocks);
}

}  // namespace

template <typename K>
hipError_t hisa_count_runs(const K* keys, u64 n, int shift, u64* d_runs, hipStream_t s) {
  hipError_t e = fill_zero(d_runs, sizeof(u64), s);
  if (e != hipSuccess || n == 0) return e;
  count_runs_kernel<K><<<grid_for(n, 8192), kNT, 0, s>>>(keys, n, shift, d_runs);
  return hipGetLastError();
}

template <typename K>
hipError_t hisa_build(const K* keys, u64 n, int shift, Slot* table, u64 cap, hipStream_t s,
                      LaunchTimer* timer) {
  if (n == 0) return hipSuccess;
  if (cap == 0 || cap > (u64(1) << 32)) return hipErrorInvalidValue;
  const u64 blocks = (n + kNT - 1) / kNT;
  if (blocks >= (u64(1) << 31)) return hipErrorInvalidValue;
  if (timer) timer->begin(K_HISA_BUILD, s);
  build_kernel<K><<<dim3(u32(blocks)), kNT, 0, s>>>(keys, n, shift, table, cap);
  if (timer) timer->end(K_HISA_BUILD, s, n * sizeof(K));
  return hipGetLastError();
}

hipError_t hisa_probe(const Slot* table, u64 cap, const u32* q, u64 nq, u64* start, u32* len,
                      hipStream_t s) {
  if (nq == 0) return hipSuccess;
  if (cap == 0 || cap > (u64(1) << 32)) return hipErrorInvalidValue;
  const u64 blocks = (nq + kNT - 1) / kNT;
  if (blocks >= (u64(1) << 31)) return hipErrorInvalidValue;
  probe_kernel<<<dim3(u32(blocks)), kNT, 0, s>>>(table, cap, q, nq, start, len);
  return hipGetLastError();
}

hipError_t fill_zero(void* p, u64 bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  // p is 16-byte aligned for every buffer this library zeroes
  u64 n16 = bytes / 16;
  u64 ntail = bytes - n16 * 16;
  zero_kernel<<<grid_for(n16 ? n16 : 1), kNT, 0, s>>>(
      static_cast<uint4*>(p), n16, static_cast<unsigned char*>(p) + n16 * 16, ntail);
  return hipGetLastError();
}

hipError_t max_u32(const u32* v, u64 n, u32* d_max, hipStream_t s) {
  if (n == 0) return hipSuccess;
  max_kernel<<<grid_for(n, 4096), kNT, 0, s>>>(v, n, d_max);
  return hipGetLastError();
}

template <typename K>
hipError_t pack_rows(const u32* rows, u64 n, int arity, int w, K* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  pack_kernel<K><<<grid_for(n), kNT, 0, s>>>(rows, n, arity, w, out);
  return hipGetLastError();
}

template <typename K>
hipError_t swap_cols(const K* in, u64 n, int w, K* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  swap_kernel<K><<<grid_for(n), kNT, 0, s>>>(in, n, w, out);
  return hipGetLastError();
}

template <typename K>
hipError_t unpack_rows(const K* keys, u64 n, int arity, int w, u32* rows, hipStream_t s,
                       u32 sub) {
  if (n == 0) return hipSuccess;
  unpack_kernel<K><<<grid_for(n), kNT, 0, s>>>(keys, n, arity, w, rows, sub);
  return hipGetLastError();
}

template <typename K>
hipError_t key_range(const K* keys, u64 n, K lo, K hi, u64* out, hipStream_t s) {
  key_range_kernel<K><<<1, 64, 0, s>>>(keys, n, lo, hi, out);
  return hipGetLastError();
}

#define HL_INSTANTIATE(K)                                                                    \
  template hipError_t hisa_count_runs<K>(const K*, u64, int, u64*, hipStream_t);            \
  template hipError_t hisa_build<K>(const K*, u64, int, Slot*, u64, hipStream_t,            \
                                    LaunchTimer*);                                            \
  template hipError_t pack_rows<K>(const u32*, u64, int, int, K*, hipStream_t);             \
  template hipError_t swap_cols<K>(const K*, u64, int, K*, hipStream_t);                    \
  template hipError_t unpack_rows<K>(const K*, u64, int, int, u32*, hipStream_t, u32);      \
  template hipError_t key_range<K>(const K*, u64, K, K, u64*, hipStream_t);
HL_INSTANTIATE(u32)
HL_INSTANTIATE(u64)
#undef HL_INSTANTIATE

}  // namespace hl
