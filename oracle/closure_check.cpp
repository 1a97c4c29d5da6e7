// Exact whole-relation checkers for the benchmark-sized fixpoints.
//
// TEST INFRASTRUCTURE ONLY (part of the oracle): used by tests/ and never by
// the GPU library.  It shares no code with the HIP path.
//
// Each checker decides whether a fetched relation equals its definition,
// every row included, without materialising the expected set:
//
//  * Reach (Section 1: Reach(x, y) holds iff y is reachable from x by one
//    or more Edge steps).  For every source s a breadth-first search marks
//    the nodes reachable from s; the rows of s must be strictly increasing
//    (so they are distinct), each must be marked, and their number must be
//    the number of marked nodes.  Together these give set equality per
//    source.  The search also yields the shortest-distance histogram, from
//    which the per-iteration delta sizes of semi-naive evaluation follow.
//  * Same generation on a rooted tree (Section 2: SG(x, y) holds iff x and
//    y are distinct nodes at the same depth below the root).  Every row must
//    satisfy that predicate and the rows must be strictly increasing; with
//    the closed-form count (checked by the caller) this is set equality.
//
// Rows are row-major uint32 pairs sorted lexicographically, as the library
// returns them.  Work is split over `threads` host threads.
#include <atomic>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

using u32 = uint32_t;
using u64 = uint64_t;
using i64 = int64_t;

// Runs f(t) on `threads` threads (t = 0 .. threads-1) and joins them.
template <typename F>
void parallel(int threads, F f) {
  if (threads < 1) threads = 1;
  std::vector<std::thread> ts;
  for (int t = 1; t < threads; ++t) ts.emplace_back(f, t);
  f(0);
  for (auto& th : ts) th.join();
}

struct Csr {
  std::vector<u64> off;
  std::vector<u32> dst;
};

// Adjacency lists of a directed graph; false if an id is out of range.
bool build_csr(u32 n, const u32* edges, u64 m, Csr& g) {
  g.off.assign(u64(n) + 1, 0);
  for (u64 i = 0; i < m; ++i) {
    if (edges[2 * i] >= n || edges[2 * i + 1] >= n) return false;
    ++g.off[edges[2 * i] + 1];
  }
  for (u64 v = 0; v < n; ++v) g.off[v + 1] += g.off[v];
  g.dst.resize(m);
  std::vector<u64> cur(g.off.begin(), g.off.end() - 1);
  for (u64 i = 0; i < m; ++i) g.dst[cur[edges[2 * i]]++] = edges[2 * i + 1];
  return true;
}

// Rows strictly increasing as (first, second) pairs and every id below n.
bool rows_valid(const u32* rows, u64 nr, u32 n, int threads) {
  std::atomic<bool> ok{true};
  parallel(threads, [&](int t) {
    const u64 lo = nr * u64(t) / u64(threads), hi = nr * u64(t + 1) / u64(threads);
    for (u64 i = lo; i < hi && ok.load(std::memory_order_relaxed); ++i) {
      const u32 a = rows[2 * i], b = rows[2 * i + 1];
      if (a >= n || b >= n) {
        ok = false;
        break;
      }
      if (i > 0) {
        const u32 pa = rows[2 * i - 2], pb = rows[2 * i - 1];
        if (!(pa < a || (pa == a && pb < b))) {
          ok = false;
          break;
        }
      }
    }
  });
  return ok;
}

// Per-thread state of the reachability searches.
struct Bfs {
  std::vector<u32> stamp;  // stamp[v] == s + 1: v reached from source s
  std::vector<u32> queue;
  explicit Bfs(u32 n) : stamp(n, 0), queue(n) {}

  // Marks the nodes reachable from s by >= 1 edge; returns how many, and
  // adds each one's shortest distance to hist (false if a distance does not
  // fit the histogram).
  bool run(const Csr& g, u32 s, u64* hist, int max_dist, u64* reached) {
    const u32 mark = s + 1;
    u64 head = 0, tail = 0, cnt = 0;
    for (u64 k = g.off[s]; k < g.off[u64(s) + 1]; ++k) {
      const u32 v = g.dst[k];
      if (stamp[v] != mark) {
        stamp[v] = mark;
        queue[tail++] = v;
      }
    }
    int d = 1;
    while (head < tail) {
      const u64 level_end = tail;
      if (d >= max_dist) return false;
      hist[d] += level_end - head;
      cnt += level_end - head;
      for (; head < level_end; ++head) {
        const u32 u = queue[head];
        for (u64 k = g.off[u]; k < g.off[u64(u) + 1]; ++k) {
          const u32 v = g.dst[k];
          if (stamp[v] != mark) {
            stamp[v] = mark;
            queue[tail++] = v;
          }
        }
      }
      ++d;
    }
    *reached = cnt;
    return true;
  }
};

// Checks one graph's closure against its rows.  Returns the number of
// sources whose rows differ (the smallest such source in *bad), or -1 for
// unsorted rows or ids out of range, -2 for a distance beyond max_dist.
i64 verify_reach(u32 n, const u32* edges, u64 m, const u32* rows, u64 nr, u64* hist,
                 int max_dist, int threads, i64* bad) {
  *bad = -1;
  Csr g;
  if (!build_csr(n, edges, m, g)) return -1;
  if (!rows_valid(rows, nr, n, threads)) return -1;
  // first row of each source (rows are sorted by their first column)
  std::vector<u64> first(u64(n) + 1, nr);
  parallel(threads, [&](int t) {
    const u64 lo = u64(n) * u64(t) / u64(threads), hi = u64(n) * u64(t + 1) / u64(threads);
    for (u64 s = lo; s < hi; ++s) {
      u64 a = 0, b = nr;
      while (a < b) {
        const u64 mid = (a + b) / 2;
        if (rows[2 * mid] < s) a = mid + 1;
        else b = mid;
      }
      first[s] = a;
    }
  });
  std::atomic<u64> next{0};
  std::atomic<i64> mism{0};
  std::atomic<i64> smallest{-1};
  std::atomic<bool> too_far{false};
  std::vector<std::vector<u64>> hists(threads < 1 ? 1 : threads,
                                      std::vector<u64>(max_dist, 0));
  parallel(threads, [&](int t) {
    Bfs b(n);
    u64* h = hists[t].data();
    constexpr u64 kGrain = 64;
    for (;;) {
      const u64 s0 = next.fetch_add(kGrain);
      if (s0 >= n) break;
      const u64 s1 = s0 + kGrain < n ? s0 + kGrain : n;
      for (u64 s = s0; s < s1; ++s) {
        u64 reached = 0;
        if (!b.run(g, u32(s), h, max_dist, &reached)) {
          too_far = true;
          return;
        }
        const u64 r0 = first[s], r1 = first[s + 1];
        bool same = (r1 - r0) == reached;
        for (u64 i = r0; same && i < r1; ++i)
          if (b.stamp[rows[2 * i + 1]] != u32(s) + 1) same = false;
        if (!same) {
          ++mism;
          i64 cur = smallest.load();
          while ((cur < 0 || i64(s) < cur) && !smallest.compare_exchange_weak(cur, i64(s))) {
          }
        }
      }
    }
  });
  if (too_far) return -2;
  for (int d = 0; d < max_dist; ++d) {
    u64 c = 0;
    for (auto& hh : hists) c += hh[d];
    hist[d] = c;
  }
  *bad = smallest.load();
  return mism.load();
}

}  // namespace

extern "C" {

// Reach over one graph: see verify_reach.  hist[d] receives the number of
// (source, target) pairs at shortest distance d (max_dist entries).
int64_t or_reach_verify(uint32_t n_nodes, const uint32_t* edges, uint64_t n_edges,
                        const uint32_t* rows, uint64_t n_rows, uint64_t* hist, int max_dist,
                        int threads, int64_t* bad_source) {
  if (!hist || max_dist < 2 || !bad_source) return -1;
  std::memset(hist, 0, sizeof(u64) * u64(max_dist));
  return verify_reach(n_nodes, edges, n_edges, rows, n_rows, hist, max_dist, threads,
                      bad_source);
}

// Reach over many independent graphs (instance k: nodes[k] ids, edges
// [edge_off[k], edge_off[k+1]) of `edges`, rows [row_off[k], row_off[k+1])
// of `rows`, all with instance-local ids).  Instances are spread over the
// threads, one search thread each.  Returns the number of instances whose
// rows differ (the smallest in *bad_inst), or -1 / -2 as above; hist sums
// the distance histograms of all instances.
int64_t or_reach_verify_many(uint32_t n_inst, const uint32_t* nodes, const uint64_t* edge_off,
                             const uint32_t* edges, const uint64_t* row_off,
                             const uint32_t* rows, uint64_t* hist, int max_dist, int threads,
                             int64_t* bad_inst) {
  if (!hist || max_dist < 2 || !bad_inst) return -1;
  std::memset(hist, 0, sizeof(u64) * u64(max_dist));
  *bad_inst = -1;
  std::atomic<u32> next{0};
  std::atomic<i64> mism{0}, smallest{-1}, status{0};
  std::vector<std::vector<u64>> hists(threads < 1 ? 1 : threads,
                                      std::vector<u64>(max_dist, 0));
  parallel(threads, [&](int t) {
    for (;;) {
      const u32 k = next.fetch_add(1);
      if (k >= n_inst || status.load() != 0) break;
      std::vector<u64> h(max_dist, 0);
      i64 bad = -1;
      const i64 r = verify_reach(nodes[k], edges + 2 * edge_off[k], edge_off[k + 1] - edge_off[k],
                                 rows + 2 * row_off[k], row_off[k + 1] - row_off[k], h.data(),
                                 max_dist, 1, &bad);
      if (r < 0) {
        status = r;
        break;
      }
      for (int d = 0; d < max_dist; ++d) hists[t][d] += h[d];
      if (r > 0) {
        ++mism;
        i64 cur = smallest.load();
        while ((cur < 0 || i64(k) < cur) && !smallest.compare_exchange_weak(cur, i64(k))) {
        }
      }
    }
  });
  if (status.load() != 0) return status.load();
  for (int d = 0; d < max_dist; ++d) {
    u64 c = 0;
    for (auto& hh : hists) c += hh[d];
    hist[d] = c;
  }
  *bad_inst = smallest.load();
  return mism.load();
}

// Same generation on a rooted tree given as (parent, child) edges: returns
// the number of rows that are not a pair of distinct nodes of the same depth
// below the root (depth >= 1; an id outside every edge counts as a root; the
// first such row index in *bad_row), or -1 if the rows are not strictly
// increasing, -3 if the edges do not form a rooted tree over ids < n_nodes.
int64_t or_sg_tree_verify(uint32_t n_nodes, const uint32_t* edges, uint64_t n_edges,
                          const uint32_t* rows, uint64_t n_rows, int threads, int64_t* bad_row) {
  if (!bad_row) return -1;
  *bad_row = -1;
  std::vector<i64> parent(n_nodes, -1);
  for (u64 i = 0; i < n_edges; ++i) {
    const u32 p = edges[2 * i], c = edges[2 * i + 1];
    if (p >= n_nodes || c >= n_nodes || parent[c] >= 0 || p == c) return -3;
    parent[c] = p;
  }
  // depth by walking up with memoisation (-1: not yet known)
  std::vector<i64> depth(n_nodes, -1);
  std::vector<u32> path;
  for (u32 v = 0; v < n_nodes; ++v) {
    u32 u = v;
    path.clear();
    while (depth[u] < 0 && parent[u] >= 0) {
      path.push_back(u);
      u = u32(parent[u]);
      if (path.size() > n_nodes) return -3;  // a cycle
    }
    i64 d = depth[u] < 0 ? 0 : depth[u];
    if (depth[u] < 0) depth[u] = 0;
    for (size_t k = path.size(); k-- > 0;) depth[path[k]] = ++d;
  }
  if (!rows_valid(rows, n_rows, n_nodes, threads)) return -1;
  std::atomic<i64> bad{0}, first_bad{-1};
  parallel(threads, [&](int t) {
    const u64 lo = n_rows * u64(t) / u64(threads), hi = n_rows * u64(t + 1) / u64(threads);
    i64 nb = 0, fb = -1;
    for (u64 i = lo; i < hi; ++i) {
      const u32 x = rows[2 * i], y = rows[2 * i + 1];
      if (x == y || depth[x] != depth[y] || depth[x] == 0) {
        if (fb < 0) fb = i64(i);
        ++nb;
      }
    }
    if (nb) {
      bad += nb;
      i64 cur = first_bad.load();
      while ((cur < 0 || fb < cur) && !first_bad.compare_exchange_weak(cur, fb)) {
      }
    }
  });
  *bad_row = first_bad.load();
  return bad.load();
}

}  // extern "C"
