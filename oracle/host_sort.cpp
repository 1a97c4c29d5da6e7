// Host-core side of the sort / merge / memory microbenchmark: the paper
// compares its two most expensive phases, sorting and merging tuples, and
// the allocation and initialisation of their buffers, between a 32-core
// CPU and a GPU (Section 6.6, the CPU/GPU table).  These are the host
// counterparts of the GPU library's sort and merge of 64-bit packed
// tuples, run on T threads of the host:
//   * sort: T chunks sorted with std::sort at once, then rounds of pairwise
//     merges of neighbouring runs, each round spread over the T threads by
//     output position (merge path: a thread's output range starts where the
//     diagonal search says the two inputs have contributed that many keys);
//   * merge: one such merge of two sorted arrays;
//   * memory: a fresh buffer of the tuples' size, every page written once
//     (malloc + parallel memset).
// Measurement infrastructure only (the cpu_baseline leg of bench.py): it
// shares no code with the GPU library.
#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

namespace {

using u64 = uint64_t;
using Clock = std::chrono::steady_clock;

double since(Clock::time_point t0) {
  return std::chrono::duration<double>(Clock::now() - t0).count();
}

template <typename F>
void parallel(int threads, F f) {
  std::vector<std::thread> pool;
  pool.reserve(threads);
  for (int t = 0; t < threads; ++t) pool.emplace_back(f, t);
  for (auto& th : pool) th.join();
}

// Keys of a among the first `diag` outputs of merge(a, b), ties taking a
// first.
u64 split_of(const u64* a, u64 na, const u64* b, u64 nb, u64 diag) {
  u64 lo = diag > nb ? diag - nb : 0;
  u64 hi = diag < na ? diag : na;
  while (lo < hi) {
    const u64 mid = lo + (hi - lo) / 2;
    if (b[diag - 1 - mid] < a[mid]) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// Output positions [d0, d1) of merge(a, b) into out.
void merge_range(const u64* a, u64 na, const u64* b, u64 nb, u64* out, u64 d0, u64 d1) {
  if (d0 >= d1) return;
  const u64 a0 = split_of(a, na, b, nb, d0), a1 = split_of(a, na, b, nb, d1);
  std::merge(a + a0, a + a1, b + (d0 - a0), b + (d1 - a1), out + d0);
}

}  // namespace

extern "C" {

// Sorts keys[0, n) ascending on `threads` threads, with tmp[0, n) as the
// second buffer.  Returns the seconds taken.
double or_host_sort_u64(u64* keys, u64* tmp, u64 n, int threads) {
  if (threads < 1) threads = 1;
  const auto t0 = Clock::now();
  if (n < 2) return since(t0);
  std::vector<u64> bounds;
  for (int t = 0; t <= threads; ++t) bounds.push_back(n * u64(t) / u64(threads));
  parallel(threads, [&](int t) { std::sort(keys + bounds[t], keys + bounds[t + 1]); });
  u64* src = keys;
  u64* dst = tmp;
  while (bounds.size() > 2) {
    std::vector<u64> next;
    for (size_t r = 0; r + 1 < bounds.size(); r += 2) next.push_back(bounds[r]);
    next.push_back(n);
    const std::vector<u64>& cur = bounds;
    parallel(threads, [&](int t) {
      const u64 lo = n * u64(t) / u64(threads), hi = n * u64(t + 1) / u64(threads);
      for (size_t r = 0; r + 1 < cur.size(); r += 2) {
        const u64 s0 = cur[r];
        const u64 s1 = r + 2 < cur.size() ? cur[r + 2] : cur[r + 1];
        const u64 mid = cur[r + 1];
        const u64 p0 = std::max(lo, s0), p1 = std::min(hi, s1);
        if (p0 >= p1) continue;
        if (mid >= s1) {  // an odd run out: copied through
          std::memcpy(dst + p0, src + p0, (p1 - p0) * sizeof(u64));
          continue;
        }
        merge_range(src + s0, mid - s0, src + mid, s1 - mid, dst + s0, p0 - s0, p1 - s0);
      }
    });
    bounds.swap(next);
    std::swap(src, dst);
  }
  if (src != keys) {
    parallel(threads, [&](int t) {
      const u64 lo = n * u64(t) / u64(threads), hi = n * u64(t + 1) / u64(threads);
      std::memcpy(keys + lo, src + lo, (hi - lo) * sizeof(u64));
    });
  }
  return since(t0);
}

// out[0, na + nb) = merge of ascending a and b on `threads` threads.
// Returns the seconds taken.
double or_host_merge_u64(const u64* a, u64 na, const u64* b, u64 nb, u64* out, int threads) {
  if (threads < 1) threads = 1;
  const auto t0 = Clock::now();
  const u64 n = na + nb;
  parallel(threads, [&](int t) {
    merge_range(a, na, b, nb, out, n * u64(t) / u64(threads), n * u64(t + 1) / u64(threads));
  });
  return since(t0);
}

// A fresh buffer of `bytes`, every byte written once on `threads` threads,
// then released.  Returns the seconds of the allocation and the writes, or
// a negative value if the allocation failed.
double or_host_alloc_init(u64 bytes, int threads) {
  if (threads < 1) threads = 1;
  const auto t0 = Clock::now();
  unsigned char* p = static_cast<unsigned char*>(std::malloc(bytes ? bytes : 1));
  if (!p) return -1.0;
  parallel(threads, [&](int t) {
    const u64 lo = bytes * u64(t) / u64(threads), hi = bytes * u64(t + 1) / u64(threads);
    std::memset(p + lo, 0, hi - lo);
  });
  const double s = since(t0);
  std::free(p);
  return s;
}

}  // extern "C"
