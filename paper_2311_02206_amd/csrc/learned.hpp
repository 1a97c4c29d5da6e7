// Device side of the learned position index (see learned.hip): the view a
// kernel receives and the exact windowed lower_bound.
#pragma once

#include "device.hpp"

namespace hl {

template <typename K>
struct LearnedView {
  const K* keys;    // sorted ascending
  u64 n;            // < 2^32
  int shift;        // bucket of x is x >> shift
  u32 T;            // number of buckets
  const u32* table; // T + 1 entries: table[r] = lower_bound(keys, r << shift)
  const u32* eps;   // T entries: error bound of the bucket's model
};

// Offset of x from its bucket's first position, predicted by linear
// interpolation over the bucket's key span.  Non-decreasing in x (each step
// rounds monotonically); the fit and every probe use this same function,
// with no contraction.
template <typename K>
__device__ __forceinline__ float lm_offset(K x, int shift, u32 lo, u32 hi) {
  const K base = (x >> shift) << shift;
  const float inv_span = __uint_as_float(u32(127 - shift) << 23);  // 2^-shift, exact
  const float frac = __fmul_rn(float(x - base), inv_span);
  return __fmul_rn(frac, float(hi - lo));
}

// Positions [a, b] that hold the first position whose key is >= x: the
// model's prediction widened by the bucket's error bound, clamped to the
// bucket (a == b == n when x is beyond every bucket).
template <typename K>
__device__ __forceinline__ void lm_window(const LearnedView<K>& lv, K x, u64& a, u64& b) {
  const u64 r = u64(x >> lv.shift);
  if (r >= lv.T) {
    a = b = lv.n;
    return;
  }
  const u32 lo = lv.table[r], hi = lv.table[r + 1];
  if (lo == hi) {
    a = b = lo;
    return;
  }
  const float off = lm_offset(x, lv.shift, lo, hi);
  const u64 f = u64(off);
  const u64 e = lv.eps[r];
  a = u64(lo) + (f > e ? f - e : 0);
  b = u64(lo) + f + e + 2;
  if (b > hi) b = hi;
  if (a > b) a = b;
}

// First position whose key is >= x (n if none).
template <typename K>
__device__ __forceinline__ u32 lm_lower_bound(const LearnedView<K>& lv, K x) {
  u64 a, b;
  lm_window(lv, x, a, b);
  while (a < b) {
    const u64 mid = (a + b) >> 1;
    if (lv.keys[mid] < x) a = mid + 1;
    else b = mid;
  }
  return u32(a);
}

}  // namespace hl
