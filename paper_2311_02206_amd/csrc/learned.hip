// Learned position index over a sorted key array.  This is an addition of
// this build, not part of the paper's HISA.
//
// Model: a radix table on the top R bits of the key brackets the answer
// exactly, since table[r] = lower_bound(keys, r << shift).  Inside a bucket,
// a linear model in fp32 predicts the offset from the bucket start:
//   off(x) = float(x - (r << shift)) * 2^-shift * float(hi - lo).
// off is monotone in x.  The bucket's error bound eps is the maximum
// |off(k) - (position of k - lo)| over its keys, measured when the index is
// fitted, with the same device function.  Then lower_bound(x), for any x
// present or not, lies in
//   [lo + floor(off) - eps, lo + floor(off) + eps + 2) ∩ [lo, hi],
// and a binary search of that window is exact whatever the model's quality.
// This is the exact ±eps window probe the learned index is meant to give.
// Refitting after a merge is one pass over the array, with no atomics on a
// hash table.
#include "device.hpp"
#include "kernels.hpp"

namespace hl {

namespace {

constexpr int kNT = 256;

constexpr u32 kUnset = 0xffffffffu;
constexpr u64 kGapPerKey = 64;  // table entries one key fills at most

// table[r] = first position whose bucket is >= r.  Each key fills the
// buckets between its predecessor's and its own, up to kGapPerKey of them;
// longer gaps (head, tail, sparse regions) are left unset for the next pass.
template <typename K>
__global__ __launch_bounds__(kNT) void lm_table_kernel(const K* keys, u64 n, int shift,
                                                       u32* table) {
  const u64 i = u64(blockIdx.x) * kNT + threadIdx.x;
  if (i >= n) return;
  const u64 b = u64(keys[i] >> shift);
  const u64 pb = i == 0 ? u64(0) : u64(keys[i - 1] >> shift) + 1;
  const u64 stop = (b - pb + 1 > kGapPerKey && b >= pb) ? pb + kGapPerKey - 1 : b;
  for (u64 r = pb; r <= stop && r <= b; ++r) table[r] = u32(i);
}

// Unset entries: a binary search each (r == T is the end: n).
template <typename K>
__global__ __launch_bounds__(kNT) void lm_fill_kernel(const K* keys, u64 n, int shift, u64 T,
                                                      u32* table) {
  const u64 r = u64(blockIdx.x) * kNT + threadIdx.x;
  if (r > T) return;
  if (r == T) {
    table[r] = u32(n);
    return;
  }
  if (table[r] != kUnset) return;
  const K x = K(r) << shift;
  u64 a = 0, b = n;
  while (a < b) {
    const u64 mid = (a + b) >> 1;
    if (keys[mid] < x) a = mid + 1;
    else b = mid;
  }
  table[r] = u32(a);
}

__global__ __launch_bounds__(kNT) void lm_unset_kernel(u32* table, u64 cnt) {
  const u64 stride = u64(gridDim.x) * kNT;
  for (u64 i = u64(blockIdx.x) * kNT + threadIdx.x; i < cnt; i += stride) table[i] = kUnset;
}

// One lane per key.  Keys are sorted, so a bucket's keys are contiguous: a
// segmented max over each wave's runs of equal bucket leaves the run's
// maximum in its first lane, which alone updates eps.
template <typename K>
__global__ __launch_bounds__(kNT) void lm_eps_kernel(const K* keys, u64 n, int shift,
                                                     const u32* table, u32* eps) {
  const u64 i = u64(blockIdx.x) * kNT + threadIdx.x;
  const bool valid = i < n;
  u32 r = 0xffffffffu, e = 0;
  bool first = false;
  if (valid) {
    const K k = keys[i];
    r = u32(k >> shift);
    const u32 lo = table[r], hi = table[r + 1];
    const float off = lm_offset(k, shift, lo, hi);
    // exact: a float and an integer below 2^32 are both exact in double
    e = u32(ceil(fabs(double(off) - double(u32(i) - lo))));
    first = lane_id() == 0 || i == 0 || u32(keys[i - 1] >> shift) != r;
  }
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const u32 eo = __shfl_down(e, d, kWave);
    const u32 ro = __shfl_down(r, d, kWave);
    if (lane_id() + d < kWave && ro == r && eo > e) e = eo;
  }
  if (valid && first && e) atomicMax(&eps[r], e);
}

__global__ __launch_bounds__(kNT) void lm_query_kernel(LearnedView<u32> lv, const u32* q, u64 nq,
                                                       u32* out) {
  const u64 i = u64(blockIdx.x) * kNT + threadIdx.x;
  if (i < nq) out[i] = lm_lower_bound(lv, q[i]);
}

__global__ __launch_bounds__(kNT) void lm_query64_kernel(LearnedView<u64> lv, const u64* q,
                                                         u64 nq, u32* out) {
  const u64 i = u64(blockIdx.x) * kNT + threadIdx.x;
  if (i < nq) out[i] = lm_lower_bound(lv, q[i]);
}

}  // namespace

// About 16 to 32 keys per bucket: the table stays small and the fit makes
// few atomic updates, while a window search costs a few steps more.
int learned_bits(u64 n, int key_bits) {
  int r = 4;
  while (r < 24 && (u64(1) << (r + 4)) < n) ++r;
  return r < key_bits ? r : key_bits;
}

u64 learned_bytes(int radix_bits) {
  const u64 T = u64(1) << radix_bits;
  return align_up((T + 1) * sizeof(u32), 256) + align_up(T * sizeof(u32), 256);
}

template <typename K>
hipError_t learned_fit(const K* keys, u64 n, int key_bits, int radix_bits, void* mem,
                       hipStream_t s, LearnedView<K>* out, LaunchTimer* timer) {
  if (n >= (u64(1) << 32) || radix_bits < 1 || radix_bits > key_bits || key_bits > int(8 * sizeof(K)))
    return hipErrorInvalidValue;
  const u64 T = u64(1) << radix_bits;
  const int shift = key_bits - radix_bits;
  char* p = static_cast<char*>(mem);
  u32* table = reinterpret_cast<u32*>(p);
  u32* eps = reinterpret_cast<u32*>(p + align_up((T + 1) * sizeof(u32), 256));
  hipError_t e = fill_zero(eps, T * sizeof(u32), s);
  if (e != hipSuccess) return e;
  if (n == 0) {
    e = fill_zero(table, (T + 1) * sizeof(u32), s);
  } else {
    if (timer) timer->begin(K_LEARNED_FIT, s);
    const u64 tb = (T + 1 + kNT - 1) / kNT;
    lm_unset_kernel<<<dim3(u32(tb < 65536 ? tb : 65536)), kNT, 0, s>>>(table, T + 1);
    lm_table_kernel<K><<<dim3(u32((n + kNT - 1) / kNT)), kNT, 0, s>>>(keys, n, shift, table);
    lm_fill_kernel<K><<<dim3(u32(tb)), kNT, 0, s>>>(keys, n, shift, T, table);
    lm_eps_kernel<K><<<dim3(u32((n + kNT - 1) / kNT)), kNT, 0, s>>>(keys, n, shift, table, eps);
    if (timer) timer->end(K_LEARNED_FIT, s, 2 * n * sizeof(K) + (T + 1) * sizeof(u32));
    e = hipGetLastError();
  }
  out->keys = keys;
  out->n = n;
  out->shift = shift;
  out->T = u32(T);
  out->table = table;
  out->eps = eps;
  return e;
}

hipError_t learned_query(const LearnedView<u32>& lv, const u32* q, u64 nq, u32* out,
                         hipStream_t s) {
  if (nq == 0) return hipSuccess;
  lm_query_kernel<<<dim3(u32((nq + kNT - 1) / kNT)), kNT, 0, s>>>(lv, q, nq, out);
  return hipGetLastError();
}

hipError_t learned_query(const LearnedView<u64>& lv, const u64* q, u64 nq, u32* out,
                         hipStream_t s) {
  if (nq == 0) return hipSuccess;
  lm_query64_kernel<<<dim3(u32((nq + kNT - 1) / kNT)), kNT, 0, s>>>(lv, q, nq, out);
  return hipGetLastError();
}

template hipError_t learned_fit<u32>(const u32*, u64, int, int, void*, hipStream_t,
                                     LearnedView<u32>*, LaunchTimer*);
template hipError_t learned_fit<u64>(const u64*, u64, int, int, void*, hipStream_t,
                                     LearnedView<u64>*, LaunchTimer*);

}  // namespace hl
