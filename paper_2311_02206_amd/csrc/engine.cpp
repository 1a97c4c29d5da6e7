// Host side of hisalog: device memory (arena + eager buffer management),
// the rule parser and planner, the semi-naive fixpoint driver and the C ABI
// declared in include/hisalog.h.  Every step of an iteration runs in the
// gfx950 kernels of this directory; the host only sequences launches and
// reads back the few counts that size the next launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/hisalog.h"
#include "kernels.hpp"

namespace {

using hl::JoinSpec;
using hl::Slot;
using hl::u32;
using hl::u64;

struct Error {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();  // clear the sticky launch error
    fail(HL_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}
#define HIPCK(expr) hip_check((expr), #expr)

// ------------------------------------------------------------------ memory

// Device memory provider.  With a caller arena every buffer is carved out
// of it (first fit, 256-byte aligned, coalescing free list); otherwise each
// buffer is a hipMalloc, capped by the budget.
// Device memory of one engine.  Two sources:
//  * a caller-owned arena, carved first-fit with coalescing of free ranges;
//  * hipMalloc under an optional budget.  Released blocks are kept in a
//    cache and handed out again (smallest block that fits, at most twice the
//    request), because hipMalloc of tens of GB stalls the host for seconds;
//    the cache is emptied when the budget or the device would otherwise be
//    exceeded, and at destruction.  With caching off every release is a
//    hipFree (the per-iteration allocation behaviour that eager buffer
//    management removes, kept for comparison).
// Every user of the memory is on the engine's one stream, so a released
// block may be reused by later stream work without a synchronisation.
class Memory {
 public:
  void init(void* arena, u64 arena_bytes, u64 budget, hipStream_t s) {
    base_ = static_cast<char*>(arena);
    size_ = arena_bytes;
    budget_ = budget;
    stream_ = s;
    if (base_) {
      u64 start = hl::align_up(reinterpret_cast<uintptr_t>(base_), 256) -
                  reinterpret_cast<uintptr_t>(base_);
      if (start < size_) free_[start] = size_ - start;
    }
  }
  void set_caching(bool on) {
    caching_ = on;
    if (!on) trim(~u64(0));
  }

  // Returns a block of at least `bytes`; its actual size goes to *got.
  void* alloc(u64 bytes, u64* got = nullptr) {
    bytes = hl::align_up(bytes ? bytes : 1, 256);
    void* p = nullptr;
    u64 size = bytes;
    if (base_) {
      for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= bytes) {
          u64 off = it->first, sz = it->second;
          free_.erase(it);
          if (sz > bytes) free_[off + bytes] = sz - bytes;
          p = base_ + off;
          break;
        }
      }
      if (!p) fail(HL_E_NOMEM, "arena exhausted: need " + std::to_string(bytes) + " bytes, " +
                                   std::to_string(in_use_) + " in use of " +
                                   std::to_string(size_));
    } else {
      auto it = cache_.lower_bound(bytes);
      if (it != cache_.end() && it->first <= 2 * bytes) {
        size = it->first;
        p = it->second;
        cache_.erase(it);
        cached_ -= size;
        ++hits_;
      } else {
        if (budget_ && in_use_ + cached_ + bytes > budget_)
          trim(in_use_ + cached_ + bytes - budget_);
        if (budget_ && in_use_ + bytes > budget_)
          fail(HL_E_NOMEM, "device budget exceeded: need " + std::to_string(bytes) + " bytes");
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess && cached_) {
          (void)hipGetLastError();
          trim(~u64(0));
          e = hipMalloc(&p, bytes);
        }
        if (e != hipSuccess) {
          (void)hipGetLastError();
          fail(HL_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        }
        ++allocs_;
      }
    }
    live_[p] = size;
    in_use_ += size;
    peak_ = std::max(peak_, in_use_);
    if (got) *got = size;
    return p;
  }

  void release(void* p) {
    if (!p) return;
    auto it = live_.find(p);
    if (it == live_.end()) return;
    u64 bytes = it->second;
    live_.erase(it);
    in_use_ -= bytes;
    if (base_) {
      u64 off = static_cast<char*>(p) - base_;
      auto nx = free_.lower_bound(off);
      if (nx != free_.end() && off + bytes == nx->first) {
        bytes += nx->second;
        free_.erase(nx);
      }
      auto pv = free_.lower_bound(off);
      if (pv != free_.begin()) {
        --pv;
        if (pv->first + pv->second == off) {
          pv->second += bytes;
          return;
        }
      }
      free_[off] = bytes;
    } else if (caching_) {
      cache_.emplace(bytes, p);
      cached_ += bytes;
    } else {
      (void)hipStreamSynchronize(stream_);
      (void)hipFree(p);
    }
  }

  void release_all() {
    std::vector<void*> ps;
    for (auto& kv : live_) ps.push_back(kv.first);
    for (void* p : ps) release(p);
    trim(~u64(0));
  }

  u64 peak() const { return peak_; }
  u64 allocs() const { return allocs_; }
  u64 cache_hits() const { return hits_; }
  u64 held() const { return in_use_ + cached_; }
  void reset_counters() {
    peak_ = in_use_;
    allocs_ = 0;
    hits_ = 0;
  }

 private:
  // hipFree cached blocks, largest first, until `bytes` are returned.
  void trim(u64 bytes) {
    if (cache_.empty()) return;
    (void)hipStreamSynchronize(stream_);
    u64 done = 0;
    while (!cache_.empty() && done < bytes) {
      auto it = std::prev(cache_.end());
      (void)hipFree(it->second);
      done += it->first;
      cached_ -= it->first;
      cache_.erase(it);
    }
  }

  char* base_ = nullptr;
  u64 size_ = 0, budget_ = 0, in_use_ = 0, peak_ = 0, allocs_ = 0, hits_ = 0, cached_ = 0;
  bool caching_ = true;
  hipStream_t stream_ = nullptr;
  std::map<u64, u64> free_;
  std::multimap<u64, void*> cache_;
  std::unordered_map<void*, u64> live_;
};

struct Buf {
  void* p = nullptr;
  u64 bytes = 0;
};

// Times launches with HIP events on the engine's stream.
class EventTimer : public hl::LaunchTimer {
 public:
  struct Total {
    u64 launches = 0;
    double ms = 0;
    u64 bytes = 0;
  };
  void begin(int kernel, hipStream_t s) override {
    hipEvent_t a = get();
    (void)hipEventRecord(a, s);
    open_.push_back({kernel, a, nullptr, 0, -1});
  }
  void end(int kernel, hipStream_t s, u64 bytes, const u64* dev) override {
    hipEvent_t b = get();
    (void)hipEventRecord(b, s);
    if (!open_.empty() && open_.back().kernel == kernel && !open_.back().b) {
      open_.back().b = b;
      open_.back().bytes = bytes;
      open_.back().slot = dev ? int(dev - dev_) : -1;
    }
  }
  // A zeroed device counter for the launch about to be timed, or null when
  // every counter of this collection period is taken (the launch then
  // counts its host-known bytes only).
  u64* device_counter(hipStream_t s) override {
    if (!dev_) {
      if (hipMalloc(&dev_, kSlots * sizeof(u64)) != hipSuccess) {
        (void)hipGetLastError();
        dev_ = nullptr;
        return nullptr;
      }
    }
    if (slots_used_ == kSlots) return nullptr;
    u64* c = dev_ + slots_used_++;
    if (hl::fill_zero(c, sizeof(u64), s) != hipSuccess) fail(HL_E_DEVICE, "fill_zero failed");
    return c;
  }
  // After a synchronisation of the stream.
  void collect() {
    if (slots_used_ > 0) {
      if (hipMemcpy(host_, dev_, slots_used_ * sizeof(u64), hipMemcpyDeviceToHost) != hipSuccess)
        fail(HL_E_DEVICE, "kernel byte counters could not be read");
    }
    for (const Rec& r : open_) {
      if (!r.b) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        Total& t = totals[r.kernel];
        ++t.launches;
        t.ms += ms;
        t.bytes += r.bytes + (r.slot >= 0 ? host_[r.slot] : 0);
      }
    }
    open_.clear();
    used_ = 0;
    slots_used_ = 0;
  }
  void reset() {
    open_.clear();
    used_ = 0;
    slots_used_ = 0;
    for (Total& t : totals) t = Total{};
  }
  ~EventTimer() override {
    for (hipEvent_t ev : pool_) (void)hipEventDestroy(ev);
    if (dev_) (void)hipFree(dev_);
  }
  Total totals[hl::K_COUNT];

 private:
  static constexpr int kSlots = 1024;
  struct Rec {
    int kernel;
    hipEvent_t a, b;
    u64 bytes;
    int slot;
  };
  u64* dev_ = nullptr;
  u64 host_[kSlots] = {};
  int slots_used_ = 0;
  hipEvent_t get() {
    if (used_ == pool_.size()) {
      hipEvent_t ev;
      if (hipEventCreate(&ev) != hipSuccess) fail(HL_E_DEVICE, "hipEventCreate failed");
      pool_.push_back(ev);
    }
    return pool_[used_++];
  }
  std::vector<hipEvent_t> pool_;
  size_t used_ = 0;
  std::vector<Rec> open_;
};

// ------------------------------------------------------------------ program

// The second column of a unary relation holds the constant 0: its atoms
// take this id there, which no variable has.
constexpr int kZeroVar = -2;

struct Atom {
  int rel = -1;
  int n = 0;                      // arity
  int arg[4] = {-1, -1, -1, -1};  // variable ids; wildcards get fresh ids
};

struct Rule {
  Atom head;
  std::vector<Atom> body;
  std::vector<std::pair<int, int>> neq;  // variable pairs that must differ
  int nvars = 0;
  std::string text;
};

// One binary join of a chain (Section 5.2): the carried pair (outer) is
// joined with the HISA of `inner_rel` keyed by column `inner_col`.
struct Step {
  int inner_rel = -1;
  int inner_col = 0;
  JoinSpec js{};
};

struct Plan {
  int rule = -1;
  int head = -1;
  int outer_rel = -1;
  bool outer_delta = false;
  JoinSpec proj{};          // for a body of one atom
  std::vector<Step> steps;  // empty: projection only
};

// A chain of joins over relations of arity up to 4 (wide plans): the
// carried tuple holds up to 4 live variables, and each join probes an index
// of its inner relation on every column it shares with the carried tuple.
struct WStep {
  int inner_rel = -1;
  int ix = -1;  // into rels[inner_rel].widx
  hl::WideSpec ws{};
};

struct WPlan {
  int rule = -1;
  int head = -1;
  int outer_rel = -1;
  bool outer_delta = false;
  hl::WideSpec proj{};       // for a body of one atom (proj.ai == 0)
  std::vector<WStep> steps;  // empty: projection only
  int max_cols = 0;          // widest carried tuple
};

struct Index {
  bool used = false;
  // indexes of relations of arity 3-4 (wide plans): column c of the index
  // tuple is column perm[c] of the relation, the first nj are the join
  // columns; an identity permutation indexes full itself
  int perm[4] = {0, 1, 2, 3};
  int nj = 1;
  bool identity = true;
  Buf keys, spare;  // column 1 only: the relation with columns swapped
  u64 n = 0;
  Buf table;
  u64 cap = 0, runs = 0;
  // learned position index (HL_FLAG_LEARNED_INDEX) over the same array
  Buf lm;
  bool lm_ok = false;
  const void* lm_keys = nullptr;
  u64 lm_n = 0;
  int lm_shift = 0;
  u32 lm_T = 0;
  const u32* lm_table = nullptr;
  const u32* lm_eps = nullptr;
  template <typename K>
  hl::LearnedView<K> view() const {
    return hl::LearnedView<K>{static_cast<const K*>(lm_keys), lm_n, lm_shift, lm_T, lm_table,
                              lm_eps};
  }
};

struct Relation {
  std::string name;
  int arity = 2;
  bool edb = false;
  Buf raw;
  u64 n_raw = 0;
  Buf full, full_spare, delta, cand;
  u64 n_full = 0, n_delta = 0, n_cand = 0;
  // share of the tiles of this relation's last set difference whose slice
  // of full was searched in global memory rather than streamed: a model of
  // full is fitted for the set difference only where such searches happen
  double lockstep_share = 0;
  Index idx[2];
  // indexes of the tail run of a relation probed as a join inner (kept as
  // two levels): tidx[0] over the tail itself, tidx[1] over its
  // column-swapped copy (tidx[1].keys)
  Index tidx[2];
  std::vector<Index> widx;  // indexes of wide plans
  std::vector<u64> delta_counts, new_counts;
  // in-tile dedup of the joins deriving this relation: on while they made
  // at least 1.5 outputs per distinct new tuple (raw_cand: this iteration's
  // outputs before filters and dedup)
  bool dedup = true;
  u64 raw_cand = 0;
  // new tuples already sorted, deduplicated and subtracted from full this
  // iteration (chunked joins, oversized candidate sets); pend_uniq sums the
  // distinct tuples of each absorbed chunk
  Buf pend[2];
  u64 n_pend = 0, pend_uniq = 0;
  // fused iterations: the next delta, the merge's partition points, and
  // the tail run of recent deltas kept beside full (ping-pong pair)
  Buf fz_next, fz_parts, fz_tail[2];
  u64 n_tail = 0;
};

// --------------------------------------------------------------- the parser

class Lexer {
 public:
  explicit Lexer(const std::string& s) : s_(s) {}
  void skip() {
    for (;;) {
      while (i_ < s_.size() && isspace(static_cast<unsigned char>(s_[i_]))) ++i_;
      if (i_ < s_.size() && (s_[i_] == '#' || (s_[i_] == '/' && i_ + 1 < s_.size() &&
                                               s_[i_ + 1] == '/'))) {
        while (i_ < s_.size() && s_[i_] != '\n') ++i_;
        continue;
      }
      return;
    }
  }
  bool done() {
    skip();
    return i_ >= s_.size();
  }
  bool accept(const char* lit) {
    skip();
    size_t n = strlen(lit);
    if (s_.compare(i_, n, lit) == 0) {
      i_ += n;
      return true;
    }
    return false;
  }
  void expect(const char* lit) {
    if (!accept(lit)) fail(HL_E_INVALID, std::string("parse error: expected '") + lit +
                                             "' at offset " + std::to_string(i_));
  }
  std::string ident() {
    skip();
    size_t b = i_;
    if (i_ < s_.size() && (isalpha(static_cast<unsigned char>(s_[i_])) || s_[i_] == '_')) {
      ++i_;
      while (i_ < s_.size() && (isalnum(static_cast<unsigned char>(s_[i_])) || s_[i_] == '_'))
        ++i_;
    }
    if (b == i_) fail(HL_E_INVALID, "parse error: expected a name at offset " + std::to_string(i_));
    return s_.substr(b, i_ - b);
  }
  size_t pos() const { return i_; }
  void seek(size_t p) { i_ = p; }

 private:
  const std::string& s_;
  size_t i_ = 0;
};

}  // namespace

// ------------------------------------------------------------------ engine

struct hl_engine {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  u32 flags = 0;
  float ebm_k = 8.0f;
  float load_factor = 0.5f;
  int sort_chunk_log2 = 0;  // 0: the largest one sort takes (chunk_keys)
  u32 fused_capacity = 0;  // 0: the largest that fits
  int join_items = 8;      // join expand outputs per thread (4, 8, 16)
  int sort_items = 32;     // radix sort keys per thread of a tile (16, 32)
  int diff_items = 16;     // set difference candidates per thread of a tile (8, 16)
  Memory mem;
  std::string err;

  std::vector<Relation> rels;
  std::vector<Rule> rules;
  // batch layout: instance k owns ids [base[k], base[k+1]) of the shared id
  // space (empty: no batch)
  std::vector<u64> batch_base;
  std::vector<u32> batch_rows_tmp;
  std::vector<Plan> plans0, plansR;  // iteration 0 / recursive plans
  // programs with relations of arity 3-4: wide plans instead
  bool wide = false;
  std::vector<WPlan> wplans0, wplansR;
  // per rule of the program, over the last run's non-fused iterations: the
  // outputs of its last join (its candidates before filters) and of its
  // earlier joins (the materialised intermediate results)
  std::vector<u64> rule_out, rule_mid;
  // this device's address of the static scratch of hl_sort_keys_noalloc
  void* noalloc = nullptr;
  bool ran = false;

  // run state
  int w = 1;
  int key_bytes = 4;
  Buf alt, tmp[2], ws, join_start, join_len, join_off, join_parts, rows, grp[2], jchunk;
  u64* d_small = nullptr;  // device scalars
  u64* h_small = nullptr;  // pinned mirror
  static constexpr int kSmall = 512;
  static constexpr int kChunkSlots = kSmall - 4;  // scratch words for chunked deltas
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, hipEvent_t>> marks;
  hl_stats st{};
  u64 reuses = 0;
  // fused small iterations (HL_FLAG_FUSED / HL_FLAG_HIP_GRAPH)
  u64* d_fz = nullptr;  // hl::kFusedCountWords device words
  u64* h_fz = nullptr;  // pinned mirror
  bool fz_plans = false;           // the recursive plans qualify
  bool fz_live = false;            // device counts carry over from the last iteration
  int fz_key_bytes = 0;            // key width the LDS capacities were set for
  u32 fz_cap_c = 0, fz_cap_t = 0;  // LDS capacities in keys: a joining workgroup
  u32 fz_cap_b = 0;                // the finishing workgroup: new tuples per iteration
  u64 fz_fail_at = ~u64(0);        // smallest total delta that overflowed in this run
  u64 last_in = 0, last_out = 0;   // last iteration: outer delta tuples, join outputs
  struct FzGraph {
    std::vector<unsigned char> key;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<FzGraph> fz_graphs;
  Buf fz_scratch;  // per-workgroup runs of the fused launch
  u64 fz_iterations = 0, fz_captures = 0, fz_overflows = 0;
  EventTimer ktimer;
  hl::LaunchTimer* kt() { return (flags & HL_FLAG_KERNEL_TIMING) ? &ktimer : nullptr; }
  bool learned() const { return flags & HL_FLAG_LEARNED_INDEX; }
  // ---------------------------------------------------------------- utils

  int find(const std::string& n) const {
    for (size_t k = 0; k < rels.size(); ++k)
      if (rels[k].name == n) return int(k);
    return -1;
  }
  int find_or_fail(const char* n) const {
    if (!n) fail(HL_E_INVALID, "null relation name");
    int k = find(n);
    if (k < 0) fail(HL_E_INVALID, std::string("unknown relation ") + n);
    return k;
  }

  void sync() {
    HIPCK(hipStreamSynchronize(stream));
    if (flags & HL_FLAG_KERNEL_TIMING) ktimer.collect();
  }

  // Eager buffer management (Section 5.3): a buffer that is large enough is
  // reused; one that must grow is reallocated to `want` (>= need) bytes.
  // With HL_FLAG_NO_EBM every request gets an exact-size buffer.
  void reserve(Buf& b, u64 need, u64 want) {
    if (need == 0) return;
    bool no_ebm = flags & HL_FLAG_NO_EBM;
    if (!no_ebm && b.bytes >= need) {
      ++reuses;
      return;
    }
    if (no_ebm && b.bytes == need) {
      ++reuses;
      return;
    }
    mem.release(b.p);
    b.p = nullptr;
    b.bytes = 0;
    u64 sz = no_ebm ? need : std::max(need, want);
    b.p = mem.alloc(sz, &b.bytes);
  }
  void reserve_grow(Buf& b, u64 need) { reserve(b, need, need + need / 2); }
  // Largest array of keys one sort takes (a chunk), in bytes.
  u64 chunk_bytes() const { return chunk_keys() * key_bytes; }
  // Tiles of a set difference over m candidates.
  u64 diff_tiles(u64 m) const {
    const u64 t = 256 * u64(diff_items);
    return std::max<u64>(1, (m + t - 1) / t);
  }
  // Keys of one sort chunk: 2^sort_chunk_log2 when set, else just under
  // the sort's 2^32 limit for 4-byte keys (a 17 GB chunk) and 2^31 for
  // 8-byte keys (a chunk's three buffers of 17 GB each).
  u64 chunk_keys() const {
    if (sort_chunk_log2) return u64(1) << sort_chunk_log2;
    return key_bytes == 4 ? (u64(1) << 32) - (u64(1) << 16) : u64(1) << 31;
  }
  // Like reserve_grow for a buffer that holds at most one chunk of keys in
  // its steady use: its growth stops at the chunk's size.
  void reserve_chunk(Buf& b, u64 need) {
    reserve(b, need, std::max(need, std::min(need + need / 2, chunk_bytes())));
  }
  // Like reserve_grow, but keeps the first `used` bytes of the buffer; the
  // growth stops at `limit` bytes (the candidate buffer: one chunk).
  void reserve_keep(Buf& b, u64 used, u64 need, u64 limit = ~u64(0)) {
    if (need <= b.bytes && !(flags & HL_FLAG_NO_EBM)) {
      ++reuses;
      return;
    }
    if (need <= b.bytes && b.bytes == need) {
      ++reuses;
      return;
    }
    Buf nb;
    const u64 sz =
        (flags & HL_FLAG_NO_EBM) ? need : std::max(need, std::min(need + need / 2, limit));
    nb.p = mem.alloc(sz, &nb.bytes);
    if (used) HIPCK(hipMemcpyAsync(nb.p, b.p, used, hipMemcpyDeviceToDevice, stream));
    drop(b);
    b = nb;
  }
  void drop(Buf& b) {
    mem.release(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }

  void mark(int phase) {
    if (ev_used == ev_pool.size()) {
      hipEvent_t ev;
      HIPCK(hipEventCreate(&ev));
      ev_pool.push_back(ev);
    }
    hipEvent_t ev = ev_pool[ev_used++];
    HIPCK(hipEventRecord(ev, stream));
    marks.push_back({phase, ev});
  }
  // After a synchronisation: attributes the time between marks to phases.
  void collect() {
    for (size_t k = 1; k < marks.size(); ++k) {
      int ph = marks[k - 1].first;
      if (ph < 0) continue;
      float ms = 0.f;
      HIPCK(hipEventElapsedTime(&ms, marks[k - 1].second, marks[k].second));
      st.phase_ms[ph] += ms;
    }
    if (!marks.empty()) {
      auto last = marks.back();
      marks.clear();
      // keep the last event as the start of the next segment
      std::swap(ev_pool[0], ev_pool[ev_used - 1]);
      marks.push_back({last.first, ev_pool[0]});
      ev_used = 1;
    }
  }

  // --------------------------------------------------------------- parse

  Atom parse_atom(Lexer& lx, std::map<std::string, int>& vars, int& nvars, bool head) {
    Atom a;
    std::string name = lx.ident();
    a.rel = find(name);
    if (a.rel < 0) fail(HL_E_INVALID, "undeclared relation " + name);
    lx.expect("(");
    int k = 0;
    for (;;) {
      std::string v = lx.ident();
      if (k >= 4) fail(HL_E_INVALID, "too many arguments for " + name);
      if (v == "_") {
        if (head) fail(HL_E_INVALID, "wildcard in a rule head");
        a.arg[k] = nvars++;
      } else {
        auto it = vars.find(v);
        if (it == vars.end()) it = vars.emplace(v, nvars++).first;
        a.arg[k] = it->second;
      }
      ++k;
      if (lx.accept(",")) continue;
      lx.expect(")");
      break;
    }
    if (k != rels[a.rel].arity) fail(HL_E_INVALID, "arity mismatch for " + name);
    a.n = k;
    // binary plans store a unary tuple x as the pair (x, 0)
    if (k == 1) a.arg[1] = kZeroVar;
    return a;
  }

  std::vector<Rule> parse(const std::string& text) {
    Lexer lx(text);
    std::vector<Rule> out;
    while (!lx.done()) {
      Rule r;
      size_t begin = lx.pos();
      std::map<std::string, int> vars;
      r.head = parse_atom(lx, vars, r.nvars, true);
      if (rels[r.head.rel].edb) fail(HL_E_INVALID, "rule head is an EDB relation");
      lx.expect(":-");
      std::vector<std::pair<std::string, std::string>> filters;
      for (;;) {
        size_t save = lx.pos();
        std::string id = lx.ident();
        if (lx.accept("!=")) {
          filters.push_back({id, lx.ident()});
        } else {
          lx.seek(save);
          r.body.push_back(parse_atom(lx, vars, r.nvars, false));
        }
        if (lx.accept(",")) continue;
        lx.expect(".");
        break;
      }
      std::set<int> bodyvars;
      for (auto& a : r.body)
        for (int k = 0; k < a.n; ++k) bodyvars.insert(a.arg[k]);
      for (int k = 0; k < r.head.n; ++k)
        if (const int v = r.head.arg[k]; !bodyvars.count(v))
          fail(HL_E_INVALID, "head variable not bound in the body");
      for (auto& f : filters) {
        auto a = vars.find(f.first), b = vars.find(f.second);
        if (a == vars.end() || b == vars.end() || !bodyvars.count(a->second) ||
            !bodyvars.count(b->second))
          fail(HL_E_INVALID, "filter on a variable that no body atom binds");
        r.neq.push_back({a->second, b->second});
      }
      if (r.body.empty()) fail(HL_E_INVALID, "rule without a body");
      r.text = text.substr(begin, lx.pos() - begin);
      out.push_back(r);
    }
    return out;
  }

  // ---------------------------------------------------------------- plan

  // Chain of binary joins starting from body atom `first` (Section 5.2,
  // temporarily materialised n-way joins).  The carried pair holds at most
  // two live variables; each further atom must share a variable with it.
  Plan plan_rule(int rule_id, int first, bool outer_delta) {
    const Rule& r = rules[rule_id];
    Plan p;
    p.rule = rule_id;
    p.head = r.head.rel;
    p.outer_rel = r.body[first].rel;
    p.outer_delta = outer_delta;
    auto unsupported = [&](const std::string& why) {
      fail(HL_E_UNSUPPORTED, "rule '" + r.text + "': " + why);
    };
    int cur[2] = {r.body[first].arg[0], r.body[first].arg[1]};
    // a variable repeated in the outer atom: the two columns must be equal
    int eq0 = (cur[0] == cur[1]) ? 0 : -1, eq1 = (cur[0] == cur[1]) ? 1 : -1;
    std::vector<int> remaining;
    for (int j = 0; j < int(r.body.size()); ++j)
      if (j != first) remaining.push_back(j);
    std::vector<bool> applied(r.neq.size(), false);
    auto src_of = [&](int v, const int* avail, int navail) {
      if (v == kZeroVar) return 3;  // a unary head's constant column
      for (int k = 0; k < navail; ++k)
        if (avail[k] == v) return k;
      return -1;
    };
    auto take_filter = [&](JoinSpec& js, const int* avail, int navail) {
      js.fa = js.fb = -1;
      for (size_t f = 0; f < r.neq.size(); ++f) {
        if (applied[f]) continue;
        int a = src_of(r.neq[f].first, avail, navail), b = src_of(r.neq[f].second, avail, navail);
        if (a < 0 || b < 0) continue;
        if (js.fa >= 0) unsupported("two filters apply at one join");
        js.fa = a;
        js.fb = b;
        applied[f] = true;
      }
    };
    // joins and equality tests never use the constant column
    auto in_cur = [&](int v) { return v != kZeroVar && (v == cur[0] || v == cur[1]); };
    if (remaining.empty()) {
      p.proj.outer_col = 0;
      take_filter(p.proj, cur, 2);
      p.proj.ea = eq0;
      p.proj.eb = eq1;
      p.proj.src0 = src_of(r.head.arg[0], cur, 2);
      p.proj.src1 = src_of(r.head.arg[1], cur, 2);
      return p;
    }
    while (!remaining.empty()) {
      int pick = -1;
      for (size_t q = 0; q < remaining.size() && pick < 0; ++q) {
        const Atom& b = r.body[remaining[q]];
        if (in_cur(b.arg[0]) || in_cur(b.arg[1])) pick = int(q);
      }
      if (pick < 0) unsupported("a body atom shares no variable with the carried pair");
      const Atom& b = r.body[remaining[pick]];
      remaining.erase(remaining.begin() + pick);
      Step s;
      s.inner_rel = b.rel;
      // probe on a bound column; the other column is new, or bound (then it
      // must equal its carried value), or the same variable again
      const int shared = in_cur(b.arg[0]) ? 0 : 1;
      s.inner_col = shared;
      const int sv = b.arg[shared], other = b.arg[1 - shared];
      s.js.outer_col = (cur[0] == sv) ? 0 : 1;
      int avail[3] = {cur[0], cur[1], other};
      take_filter(s.js, avail, 3);
      s.js.ea = eq0;
      s.js.eb = eq1;
      eq0 = eq1 = -1;
      if (in_cur(other)) {
        if (s.js.ea >= 0) unsupported("two equality tests apply at one join");
        s.js.ea = src_of(other, avail, 2);
        s.js.eb = 2;
      }
      if (remaining.empty()) {
        s.js.src0 = src_of(r.head.arg[0], avail, 3);
        s.js.src1 = src_of(r.head.arg[1], avail, 3);
        if (s.js.src0 < 0 || s.js.src1 < 0) unsupported("head variable lost");
      } else {
        std::set<int> need;
        for (int q : remaining) need.insert({r.body[q].arg[0], r.body[q].arg[1]});
        need.insert({r.head.arg[0], r.head.arg[1]});
        for (size_t f = 0; f < r.neq.size(); ++f)
          if (!applied[f]) need.insert({r.neq[f].first, r.neq[f].second});
        need.erase(kZeroVar);
        std::vector<int> keep;
        for (int k = 0; k < 3; ++k)
          if (need.count(avail[k]) && std::find(keep.begin(), keep.end(), avail[k]) == keep.end())
            keep.push_back(avail[k]);
        if (keep.size() > 2) unsupported("three variables stay live between joins");
        if (keep.empty()) unsupported("no variable carried to the next join");
        if (keep.size() == 1) keep.push_back(keep[0]);
        s.js.src0 = src_of(keep[0], avail, 3);
        s.js.src1 = src_of(keep[1], avail, 3);
        cur[0] = keep[0];
        cur[1] = keep[1];
      }
      p.steps.push_back(s);
    }
    for (size_t f = 0; f < applied.size(); ++f)
      if (!applied[f]) unsupported("a filter was never applicable");
    return p;
  }

  // ------------------------------------------------- wide plans
  // Programs with a relation of arity 3 or 4 (the paper's requirement R3,
  // Section 3): every join probes an index of its inner relation on all the
  // columns it shares with the carried tuple (a key of several columns,
  // Section 5.1), and the carried tuple holds up to 4 live variables.

  // Index of relation `rel` with columns perm[0..a) and nj join columns
  // (added if new).
  int wide_index(int rel, const int* perm, int a, int nj) {
    Relation& R = rels[rel];
    for (size_t k = 0; k < R.widx.size(); ++k) {
      const Index& ix = R.widx[k];
      if (ix.nj == nj && std::equal(perm, perm + a, ix.perm)) return int(k);
    }
    Index ix;
    ix.used = true;
    ix.nj = nj;
    ix.identity = true;
    for (int c = 0; c < 4; ++c) ix.perm[c] = c < a ? perm[c] : c;
    for (int c = 0; c < a; ++c) ix.identity = ix.identity && perm[c] == c;
    R.widx.push_back(ix);
    return int(R.widx.size()) - 1;
  }

  WPlan plan_rule_wide(int rule_id, int first, bool outer_delta) {
    const Rule& r = rules[rule_id];
    WPlan p;
    p.rule = rule_id;
    p.head = r.head.rel;
    p.outer_rel = r.body[first].rel;
    p.outer_delta = outer_delta;
    auto unsupported = [&](const std::string& why) {
      fail(HL_E_UNSUPPORTED, "rule '" + r.text + "': " + why);
    };
    const Atom& a0 = r.body[first];
    // the carried tuple: the variable of each of its columns
    std::vector<int> cur(a0.arg, a0.arg + a0.n);
    p.max_cols = a0.n;
    // a variable repeated in the outer atom: its columns must be equal
    std::vector<std::pair<int, int>> eqs;
    for (int i = 0; i < a0.n; ++i)
      for (int j = 0; j < i; ++j)
        if (cur[i] == cur[j]) {
          eqs.push_back({j, i});
          break;
        }
    std::vector<bool> applied(r.neq.size(), false);
    auto src_of = [](int v, const std::vector<int>& carried, const std::vector<int>& inner) {
      for (size_t k = 0; k < carried.size(); ++k)
        if (carried[k] == v) return int(k);
      for (size_t k = 0; k < inner.size(); ++k)
        if (inner[k] == v) return 4 + int(k);
      return -1;
    };
    auto add_filters = [&](hl::WideSpec& ws, const std::vector<int>& carried,
                           const std::vector<int>& inner) {
      for (size_t f = 0; f < r.neq.size(); ++f) {
        if (applied[f]) continue;
        const int a = src_of(r.neq[f].first, carried, inner);
        const int b = src_of(r.neq[f].second, carried, inner);
        if (a < 0 || b < 0) continue;
        if (ws.nf >= 4) unsupported("more than four filters apply at one join");
        ws.fa[ws.nf] = a;
        ws.fb[ws.nf] = b;
        ++ws.nf;
        applied[f] = true;
      }
    };
    auto add_eq = [&](hl::WideSpec& ws, int a, int b) {
      if (ws.ne >= 4) unsupported("more than four equality tests apply at one join");
      ws.ea[ws.ne] = a;
      ws.eb[ws.ne] = b;
      ++ws.ne;
    };
    auto set_out = [&](hl::WideSpec& ws, const std::vector<int>& vars,
                       const std::vector<int>& carried, const std::vector<int>& inner) {
      ws.nout = int(vars.size());
      for (size_t t = 0; t < vars.size(); ++t) {
        ws.src[t] = src_of(vars[t], carried, inner);
        if (ws.src[t] < 0) unsupported("head variable lost");
      }
    };
    auto in_cur = [&](int v) { return std::find(cur.begin(), cur.end(), v) != cur.end(); };
    const std::vector<int> head(r.head.arg, r.head.arg + r.head.n);
    std::vector<int> remaining;
    for (int j = 0; j < int(r.body.size()); ++j)
      if (j != first) remaining.push_back(j);
    if (remaining.empty()) {
      hl::WideSpec& ws = p.proj;
      ws.ao = a0.n;
      for (auto& e : eqs) add_eq(ws, e.first, e.second);
      add_filters(ws, cur, {});
      set_out(ws, head, cur, {});
    }
    while (!remaining.empty()) {
      // the atom sharing the most variables with the carried tuple
      int pick = -1, best = 0;
      for (size_t q = 0; q < remaining.size(); ++q) {
        const Atom& b = r.body[remaining[q]];
        std::set<int> shared;
        for (int k = 0; k < b.n; ++k)
          if (in_cur(b.arg[k])) shared.insert(b.arg[k]);
        if (int(shared.size()) > best) {
          best = int(shared.size());
          pick = int(q);
        }
      }
      // no atom shares a variable: a cross product with the first of them
      // (an index with no join columns; every outer tuple takes all of it)
      if (pick < 0) pick = 0;
      const Atom& b = r.body[remaining[pick]];
      remaining.erase(remaining.begin() + pick);
      // join columns first (every column whose variable is carried), then
      // the others, each group in atom order
      int perm[4] = {0, 1, 2, 3}, np = 0;
      for (int k = 0; k < b.n; ++k)
        if (in_cur(b.arg[k])) perm[np++] = k;
      const int nj = np;
      for (int k = 0; k < b.n; ++k)
        if (!in_cur(b.arg[k])) perm[np++] = k;
      WStep st;
      st.inner_rel = b.rel;
      st.ix = wide_index(b.rel, perm, b.n, nj);
      hl::WideSpec& ws = st.ws;
      ws.ao = int(cur.size());
      ws.ai = b.n;
      ws.nj = nj;
      std::vector<int> inner(b.n);
      for (int c = 0; c < b.n; ++c) inner[c] = b.arg[perm[c]];
      for (int t = 0; t < nj; ++t) ws.jo[t] = src_of(inner[t], cur, {});
      for (auto& e : eqs) add_eq(ws, e.first, e.second);
      eqs.clear();
      // a new variable repeated in the inner atom: its columns must be equal
      for (int c = nj; c < b.n; ++c)
        for (int c2 = nj; c2 < c; ++c2)
          if (inner[c] == inner[c2]) {
            add_eq(ws, 4 + c2, 4 + c);
            break;
          }
      add_filters(ws, cur, inner);
      if (remaining.empty()) {
        set_out(ws, head, cur, inner);
      } else {
        std::set<int> need(head.begin(), head.end());
        for (int q : remaining)
          for (int k = 0; k < r.body[q].n; ++k) need.insert(r.body[q].arg[k]);
        for (size_t f = 0; f < r.neq.size(); ++f)
          if (!applied[f]) need.insert({r.neq[f].first, r.neq[f].second});
        std::vector<int> keep;
        for (const std::vector<int>* side : {&cur, &inner})
          for (int v : *side)
            if (need.count(v) && std::find(keep.begin(), keep.end(), v) == keep.end())
              keep.push_back(v);
        if (keep.size() > 4) unsupported("more than four variables stay live between joins");
        // the joins so far only need to be non-empty: carry one variable
        // (any; the head takes none of them)
        if (keep.empty()) keep.push_back(cur[0]);
        set_out(ws, keep, cur, inner);
        cur = keep;
        p.max_cols = std::max(p.max_cols, int(keep.size()));
      }
      p.steps.push_back(st);
    }
    for (size_t f = 0; f < applied.size(); ++f)
      if (!applied[f]) unsupported("a filter was never applicable");
    return p;
  }

  void build_wide_plans() {
    for (Relation& R : rels) R.widx.clear();
    for (int k = 0; k < int(rules.size()); ++k) {
      const Rule& r = rules[k];
      bool edb_only = true;
      for (auto& a : r.body) edb_only &= rels[a.rel].edb;
      if (edb_only) {
        wplans0.push_back(plan_rule_wide(k, 0, false));
      } else {
        for (int t = 0; t < int(r.body.size()); ++t)
          if (!rels[r.body[t].rel].edb) wplansR.push_back(plan_rule_wide(k, t, true));
      }
    }
    fz_plans = false;
  }

  // Widest tuple of a wide program: relations and carried tuples.
  int wide_cols() const {
    int c = 0;
    for (const Relation& R : rels) c = std::max(c, R.arity);
    for (auto* ps : {&wplans0, &wplansR})
      for (const WPlan& p : *ps) c = std::max(c, p.max_cols);
    return c;
  }

  void build_plans() {
    plans0.clear();
    plansR.clear();
    wplans0.clear();
    wplansR.clear();
    int max_arity = 0;
    for (const Relation& R : rels) max_arity = std::max(max_arity, R.arity);
    wide = max_arity >= 3;
    if (!wide) {
      // binary chains first; a rule outside their form (three live
      // variables, a cross product) makes the whole program wide
      std::vector<std::pair<bool, bool>> used;
      for (const Relation& R : rels) used.push_back({R.idx[0].used, R.idx[1].used});
      try {
        build_binary_plans();
        return;
      } catch (const Error& x) {
        if (x.code != HL_E_UNSUPPORTED || !batch_base.empty()) throw;
        plans0.clear();
        plansR.clear();
        for (size_t k = 0; k < rels.size(); ++k) {
          rels[k].idx[0].used = used[k].first;
          rels[k].idx[1].used = used[k].second;
        }
        wide = true;
      }
    }
    if (!batch_base.empty()) fail(HL_E_UNSUPPORTED, "batches of wide programs");
    build_wide_plans();
  }

  void build_binary_plans() {
    for (int k = 0; k < int(rules.size()); ++k) {
      const Rule& r = rules[k];
      bool edb_only = true;
      for (auto& a : r.body) edb_only &= rels[a.rel].edb;
      if (edb_only) {
        plans0.push_back(plan_rule(k, 0, false));
      } else {
        for (int t = 0; t < int(r.body.size()); ++t)
          if (!rels[r.body[t].rel].edb) plansR.push_back(plan_rule(k, t, true));
      }
    }
    for (auto* ps : {&plans0, &plansR})
      for (auto& p : *ps)
        for (auto& s : p.steps) rels[s.inner_rel].idx[s.inner_col].used = true;
    // fused iterations: every inner of the recursive rules is an EDB index
    // (built once), so an iteration touches no index of its own outputs
    int idb = 0;
    for (auto& R : rels) idb += R.edb ? 0 : 1;
    fz_plans = idb >= 1 && idb <= hl::kFusedMaxRels && !plansR.empty() &&
               plansR.size() <= size_t(hl::kFusedMaxPlans);
    for (auto& p : plansR) {
      fz_plans &= p.outer_delta && p.steps.size() <= size_t(hl::kFusedMaxSteps);
      for (auto& s : p.steps) fz_plans &= rels[s.inner_rel].edb;
    }
  }

  // ----------------------------------------------------------------- run

  template <typename K>
  K* kp(Buf& b) {
    return static_cast<K*>(b.p);
  }

  template <typename K>
  void build_index(Relation& R, int col, u64* d_runs) {
    Index& ix = R.idx[col];
    const K* keys;
    if (col == 0) {
      keys = kp<K>(R.full);
      ix.n = R.n_full;
    } else {
      keys = kp<K>(ix.keys);
    }
    HIPCK(hl::hisa_count_runs<K>(keys, ix.n, w, d_runs, stream));
  }

  // Significant bits of R's packed tuples.
  int kbits(const Relation& R) const { return (wide ? R.arity : 2) * w; }

  template <typename K>
  void fit_model(Relation& R, int col) {
    Index& ix = R.idx[col];
    if (col == 0) ix.n = R.n_full;
    fit_index_model<K>(R, ix, col == 0 ? kp<K>(R.full) : kp<K>(ix.keys));
  }

  // Learned model of index ix of R over its n sorted keys.
  template <typename K>
  void fit_index_model(Relation& R, Index& ix, const K* keys) {
    ix.lm_ok = false;
    if (ix.n >= (u64(1) << 32)) {
      // positions are 32-bit: a join inner this large is unsupported, a
      // model only used by the set difference is skipped (binary search)
      if (ix.used) fail(HL_E_UNSUPPORTED, "indexed relation " + R.name +
                                              " has 2^32 or more tuples");
      return;
    }
    const int bits = hl::learned_bits(ix.n, kbits(R));
    const u64 bytes = hl::learned_bytes(bits);
    reserve(ix.lm, bytes, 2 * bytes);  // the table doubles as the relation grows
    hl::LearnedView<K> v{};
    HIPCK(hl::learned_fit<K>(keys, ix.n, kbits(R), bits, ix.lm.p, stream, &v, kt()));
    ix.lm_keys = v.keys;
    ix.lm_n = v.n;
    ix.lm_shift = v.shift;
    ix.lm_T = v.T;
    ix.lm_table = v.table;
    ix.lm_eps = v.eps;
    ix.lm_ok = true;
  }

  template <typename K>
  void finish_index(Relation& R, int col, u64 runs) {
    Index& ix = R.idx[col];
    ix.runs = runs;
    if (ix.n == 0) {
      ix.cap = 0;
      return;
    }
    if (ix.n >= (u64(1) << 32)) fail(HL_E_UNSUPPORTED, "indexed relation " + R.name +
                                                           " has 2^32 or more tuples");
    u64 cap = u64(std::ceil(double(runs) / load_factor));
    cap = std::max(cap, runs + 1);
    cap = std::max<u64>(cap, 16);
    reserve(ix.table, cap * sizeof(Slot), cap * sizeof(Slot) * 2);
    ix.cap = cap;
    HIPCK(hl::fill_zero(ix.table.p, cap * sizeof(Slot), stream));
    const K* keys = col == 0 ? kp<K>(R.full) : kp<K>(ix.keys);
    HIPCK(hl::hisa_build<K>(keys, ix.n, w, static_cast<Slot*>(ix.table.p), cap, stream, kt()));
  }

  // Refreshes every used index of the listed relations: column-1 copies
  // take the new delta (swapped, sorted, merged), then the hash tables are
  // rebuilt from the run counts (one synchronisation for all of them), or
  // the learned models refitted.  Only relations probed as join inners are
  // refreshed; the set difference uses a model when one exists (a relation
  // that is not an inner is searched directly, which costs less than a
  // refit of its whole full relation after every merge).
  template <typename K>
  void refresh_indexes(const std::vector<int>& which) {
    std::vector<std::pair<int, int>> todo;
    for (int r : which)
      for (int c = 0; c < 2; ++c)
        if (rels[r].idx[c].used) todo.push_back({r, c});
    if (todo.empty()) return;
    if (learned()) {
      // the learned index needs no run count: no synchronisation
      for (auto& rc : todo) fit_model<K>(rels[rc.first], rc.second);
      return;
    }
    if (todo.size() > kChunkSlots) fail(HL_E_UNSUPPORTED, "too many indexes");
    for (size_t q = 0; q < todo.size(); ++q) {
      Relation& R = rels[todo[q].first];
      build_index<K>(R, todo[q].second, d_small + q);
    }
    HIPCK(hipMemcpyAsync(h_small, d_small, todo.size() * sizeof(u64), hipMemcpyDeviceToHost,
                         stream));
    sync();
    for (size_t q = 0; q < todo.size(); ++q)
      finish_index<K>(rels[todo[q].first], todo[q].second, h_small[q]);
  }

  // Sorted array of wide index ix of R (full itself for the identity
  // permutation).
  template <typename K>
  const K* wide_keys(Relation& R, Index& ix) {
    return ix.identity ? kp<K>(R.full) : kp<K>(ix.keys);
  }

  // Wide index ix of R takes the new tuples src[0, n_src): permuted, sorted
  // and merged into its array (built from them when from_scratch).
  template <typename K>
  void update_wide(Relation& R, Index& ix, const K* src, u64 n_src, bool from_scratch) {
    if (ix.identity) {
      ix.n = R.n_full;
      return;
    }
    if (n_src == 0) {
      if (from_scratch) ix.n = 0;
      return;
    }
    const int bits = kbits(R);
    reserve_grow(alt, n_src * sizeof(K));
    reserve_grow(tmp[0], n_src * sizeof(K));
    HIPCK(hl::wide_permute<K>(src, n_src, R.arity, w, ix.perm, kp<K>(tmp[0]), stream));
    reserve(ws, hl::sort_workspace_bytes(n_src), hl::sort_workspace_bytes(n_src) * 2);
    K* sorted = nullptr;
    HIPCK(hl::radix_sort<K>(kp<K>(tmp[0]), kp<K>(alt), n_src, bits, ws.p, stream, &sorted, kt(),
                            sort_items));
    if (from_scratch || ix.n == 0) {
      reserve(ix.keys, n_src * sizeof(K), u64(double(n_src) * sizeof(K) * 1.5));
      HIPCK(hipMemcpyAsync(ix.keys.p, sorted, n_src * sizeof(K), hipMemcpyDeviceToDevice, stream));
      ix.n = n_src;
      return;
    }
    const u64 total = ix.n + n_src;
    reserve(ix.spare, total * sizeof(K), u64((double(ix.n) + ebm_k * double(n_src)) * sizeof(K)));
    reserve(ws, hl::merge_workspace_bytes(ix.n, n_src), hl::merge_workspace_bytes(ix.n, n_src) * 2);
    HIPCK(hl::merge<K>(kp<K>(ix.keys), ix.n, sorted, n_src, kp<K>(ix.spare), ws.p, stream, kt()));
    std::swap(ix.keys, ix.spare);
    ix.n = total;
  }

  // Hash tables (one synchronisation for the run counts of all of them) or
  // learned models of every wide index of the listed relations.
  template <typename K>
  void refresh_wide(const std::vector<int>& which) {
    std::vector<std::pair<int, int>> todo;
    for (int r : which)
      for (int k = 0; k < int(rels[r].widx.size()); ++k) todo.push_back({r, k});
    if (todo.empty()) return;
    for (auto& rk : todo) {
      Relation& R = rels[rk.first];
      Index& ix = R.widx[rk.second];
      if (ix.identity) ix.n = R.n_full;
      if (ix.n >= (u64(1) << 32))
        fail(HL_E_UNSUPPORTED, "indexed relation " + R.name + " has 2^32 or more tuples");
    }
    // an index with no join columns (a cross product's inner) is scanned
    // whole: neither a table nor a model
    todo.erase(std::remove_if(todo.begin(), todo.end(),
                              [&](const std::pair<int, int>& rk) {
                                return rels[rk.first].widx[rk.second].nj == 0;
                              }),
               todo.end());
    if (learned()) {
      for (auto& rk : todo) {
        Relation& R = rels[rk.first];
        Index& ix = R.widx[rk.second];
        fit_index_model<K>(R, ix, wide_keys<K>(R, ix));
      }
      return;
    }
    if (todo.size() > kChunkSlots) fail(HL_E_UNSUPPORTED, "too many indexes");
    for (size_t q = 0; q < todo.size(); ++q) {
      Relation& R = rels[todo[q].first];
      Index& ix = R.widx[todo[q].second];
      HIPCK(hl::wide_count_runs<K>(wide_keys<K>(R, ix), ix.n, (R.arity - ix.nj) * w,
                                   d_small + q, stream));
    }
    HIPCK(hipMemcpyAsync(h_small, d_small, todo.size() * sizeof(u64), hipMemcpyDeviceToHost,
                         stream));
    sync();
    for (size_t q = 0; q < todo.size(); ++q) {
      Relation& R = rels[todo[q].first];
      Index& ix = R.widx[todo[q].second];
      const u64 runs = h_small[q];
      ix.runs = runs;
      if (ix.n == 0) {
        ix.cap = 0;
        continue;
      }
      u64 cap = u64(std::ceil(double(runs) / load_factor));
      cap = std::max(cap, runs + 1);
      cap = std::max<u64>(cap, 16);
      reserve(ix.table, cap * sizeof(Slot), cap * sizeof(Slot) * 2);
      ix.cap = cap;
      HIPCK(hl::fill_zero(ix.table.p, cap * sizeof(Slot), stream));
      HIPCK(hl::wide_hisa_build<K>(wide_keys<K>(R, ix), ix.n, (R.arity - ix.nj) * w,
                                   static_cast<Slot*>(ix.table.p), cap, stream, kt()));
    }
  }

  // Column-1 index copy of R: merge in the swapped new delta (or build it
  // from full for an EDB relation).
  template <typename K>
  void update_swapped(Relation& R, const K* src, u64 n_src, bool from_scratch) {
    Index& ix = R.idx[1];
    if (!ix.used) return;
    if (n_src == 0) {
      if (from_scratch) ix.n = 0;
      return;
    }
    const int bits = 2 * w;
    reserve_grow(alt, n_src * sizeof(K));
    reserve_grow(tmp[0], n_src * sizeof(K));
    HIPCK(hl::swap_cols<K>(src, n_src, w, kp<K>(tmp[0]), stream));
    reserve(ws, hl::sort_workspace_bytes(n_src), hl::sort_workspace_bytes(n_src) * 2);
    K* sorted = nullptr;
    HIPCK(hl::radix_sort<K>(kp<K>(tmp[0]), kp<K>(alt), n_src, bits, ws.p, stream, &sorted, kt(),
                            sort_items));
    if (from_scratch || ix.n == 0) {
      reserve(ix.keys, n_src * sizeof(K), u64(double(n_src) * sizeof(K) * 1.5));
      HIPCK(hipMemcpyAsync(ix.keys.p, sorted, n_src * sizeof(K), hipMemcpyDeviceToDevice, stream));
      ix.n = n_src;
      return;
    }
    const u64 total = ix.n + n_src;
    reserve(ix.spare, total * sizeof(K), u64((double(ix.n) + ebm_k * double(n_src)) * sizeof(K)));
    reserve(ws, hl::merge_workspace_bytes(ix.n, n_src), hl::merge_workspace_bytes(ix.n, n_src) * 2);
    HIPCK(hl::merge<K>(kp<K>(ix.keys), ix.n, sorted, n_src, kp<K>(ix.spare), ws.p, stream, kt()));
    std::swap(ix.keys, ix.spare);
    ix.n = total;
  }

  template <typename K>
  void load_edbs() {
    std::vector<int> edbs;
    for (int k = 0; k < int(rels.size()); ++k) {
      Relation& R = rels[k];
      if (!R.edb) continue;
      edbs.push_back(k);
      R.n_full = 0;
      R.idx[0].n = R.idx[1].n = 0;
      for (Index& ix : R.widx) ix.n = ix.cap = 0;
      if (R.n_raw == 0) continue;
      if (R.n_raw >= (u64(1) << 32)) fail(HL_E_UNSUPPORTED, "EDB relation with 2^32 or more rows");
      reserve_grow(R.cand, R.n_raw * sizeof(K));
      reserve_grow(alt, R.n_raw * sizeof(K));
      if (wide)
        HIPCK(hl::wide_pack<K>(static_cast<const u32*>(R.raw.p), R.n_raw, R.arity, w,
                               kp<K>(R.cand), stream));
      else
        HIPCK(hl::pack_rows<K>(static_cast<const u32*>(R.raw.p), R.n_raw, R.arity, w,
                               kp<K>(R.cand), stream));
      reserve(ws, hl::sort_workspace_bytes(R.n_raw), hl::sort_workspace_bytes(R.n_raw) * 2);
      K* sorted = nullptr;
      HIPCK(hl::radix_sort<K>(kp<K>(R.cand), kp<K>(alt), R.n_raw, kbits(R), ws.p, stream, &sorted,
                              kt(), sort_items));
      K* other = sorted == kp<K>(R.cand) ? kp<K>(alt) : kp<K>(R.cand);
      reserve(R.full, R.n_raw * sizeof(K), R.n_raw * sizeof(K));
      reserve(ws, hl::unique_diff_workspace_bytes(R.n_raw),
              hl::unique_diff_workspace_bytes(R.n_raw) * 2);
      HIPCK(hl::unique_diff<K>(sorted, R.n_raw, static_cast<const K*>(nullptr), 0, other,
                               kp<K>(R.full), d_small, ws.p, stream, kt(), nullptr, nullptr, 0,
                               diff_items));
      HIPCK(hipMemcpyAsync(h_small, d_small, sizeof(u64), hipMemcpyDeviceToHost, stream));
      sync();
      R.n_full = h_small[0];
      R.idx[0].n = R.n_full;
      if (R.idx[1].used && !wide) update_swapped<K>(R, kp<K>(R.full), R.n_full, true);
      for (Index& ix : R.widx) update_wide<K>(R, ix, kp<K>(R.full), R.n_full, true);
    }
    if (wide) refresh_wide<K>(edbs);
    else refresh_indexes<K>(edbs);
  }

  // Evaluates one wide plan, appending head tuples to the head's
  // candidates: the same probe / scan / load-balanced expand as run_plan
  // (chunked likewise when the last join's outputs exceed one sort), with
  // keys of several columns and tuples of up to 4 columns.
  template <typename K>
  void run_wide_plan(const WPlan& p) {
    Relation& O = rels[p.outer_rel];
    const K* outer = p.outer_delta ? kp<K>(O.delta) : kp<K>(O.full);
    const u64 n = p.outer_delta ? O.n_delta : O.n_full;
    for (u64 o = 0; o < n; o += outer_slice)
      run_wide_plan_on<K>(p, outer + o, std::min(outer_slice, n - o));
  }

  template <typename K>
  void run_wide_plan_on(const WPlan& p, const K* cur, u64 n) {
    Relation& H = rels[p.head];
    if (n == 0) return;
    u64* d_cursor = d_small;
    if (p.steps.empty()) {
      hl::WideSpec ws = p.proj;
      ws.w = w;
      H.raw_cand += n;
      st.join_outputs += n;
      rule_out[p.rule] += n;
      reserve_keep(H.cand, H.n_cand * sizeof(K), (H.n_cand + n) * sizeof(K));
      const bool filtered = ws.nf > 0 || ws.ne > 0;
      if (filtered) {
        h_small[0] = H.n_cand;
        HIPCK(hipMemcpyAsync(d_cursor, h_small, sizeof(u64), hipMemcpyHostToDevice, stream));
      }
      HIPCK(hl::wide_project<K>(cur, n, ws, kp<K>(H.cand) + (filtered ? 0 : H.n_cand), d_cursor,
                                stream));
      if (filtered) {
        HIPCK(hipMemcpyAsync(h_small, d_cursor, sizeof(u64), hipMemcpyDeviceToHost, stream));
        sync();
        st.candidates += h_small[0] - H.n_cand;
        H.n_cand = h_small[0];
      } else {
        H.n_cand += n;
        st.candidates += n;
      }
      return;
    }
    int ping = 0;
    for (size_t q = 0; q < p.steps.size(); ++q) {
      const WStep& s = p.steps[q];
      Relation& I = rels[s.inner_rel];
      Index& ix = I.widx[s.ix];
      if (ix.n == 0 || (ix.nj > 0 && (learned() ? !ix.lm_ok : ix.cap == 0))) return;
      const K* inner = wide_keys<K>(I, ix);
      hl::WideSpec ws = s.ws;
      ws.w = w;
      if (n >= (u64(1) << 32)) fail(HL_E_UNSUPPORTED, "join outer side of 2^32 or more tuples");
      const bool last = q + 1 == p.steps.size();
      reserve_grow(join_start, n * sizeof(u32));
      reserve_grow(join_len, n * sizeof(u32));
      reserve_grow(join_off, n * sizeof(u64));
      if (ws.nj == 0)
        HIPCK(hl::wide_probe_all(n, ix.n, static_cast<u32*>(join_start.p),
                                 static_cast<u32*>(join_len.p), stream, kt()));
      else if (learned())
        HIPCK(hl::wide_probe_learned<K>(cur, n, ws, ix.view<K>(), static_cast<u32*>(join_start.p),
                                        static_cast<u32*>(join_len.p), stream, kt()));
      else
        HIPCK(hl::wide_probe<K>(cur, n, ws, static_cast<const Slot*>(ix.table.p), ix.cap, inner,
                                static_cast<u32*>(join_start.p), static_cast<u32*>(join_len.p),
                                stream, kt()));
      reserve(this->ws, hl::scan_workspace_bytes(n), hl::scan_workspace_bytes(n) * 2);
      HIPCK(hl::scan_u32_u64(static_cast<u32*>(join_len.p), n, static_cast<u64*>(join_off.p),
                             d_small + 1, this->ws.p, stream));
      HIPCK(hipMemcpyAsync(h_small + 1, d_small + 1, sizeof(u64), hipMemcpyDeviceToHost, stream));
      sync();
      const u64 total = h_small[1];
      if (total == 0) return;
      (last ? rule_out : rule_mid)[p.rule] += total;
      if (last) {
        H.raw_cand += total;
        st.join_outputs += total;
      }
      const bool filtered = ws.nf > 0 || ws.ne > 0;
      const u64 cap = chunk_keys();
      const u64 nt = hl::join_tiles(n, total, 8);
      reserve_grow(join_parts, hl::join_parts(n, total, 8) * sizeof(u64));
      u64* parts = static_cast<u64*>(join_parts.p);
      HIPCK(hl::join_partition(static_cast<u64*>(join_off.p), n, total, parts, stream, 8));
      if (last && total > cap) {
        // outputs beyond one sort: a range of tiles at a time, each
        // absorbed into the head's pending delta
        const u64 tile_out = hl::join_tile_outputs(8);
        const u64 per = std::max<u64>(1, cap / tile_out);
        reserve(jchunk, per * tile_out * sizeof(K), per * tile_out * sizeof(K));
        for (u64 t0 = 0; t0 < nt; t0 += per) {
          const u64 tiles = std::min(per, nt - t0);
          if (filtered) {
            h_small[0] = 0;
            HIPCK(hipMemcpyAsync(d_cursor, h_small, sizeof(u64), hipMemcpyHostToDevice, stream));
          }
          HIPCK(hl::wide_expand_tiles<K>(cur, n, static_cast<u64*>(join_off.p),
                                         static_cast<u32*>(join_start.p), inner, total, ws, parts,
                                         t0, tiles, kp<K>(jchunk), d_cursor, stream, kt()));
          u64 m;
          if (filtered) {
            HIPCK(hipMemcpyAsync(h_small, d_cursor, sizeof(u64), hipMemcpyDeviceToHost, stream));
            sync();
            m = h_small[0];
          } else {
            const u64 t1 = t0 + tiles;
            HIPCK(hipMemcpyAsync(h_small + 2, parts + t0, sizeof(u64), hipMemcpyDeviceToHost,
                                 stream));
            HIPCK(hipMemcpyAsync(h_small + 3, parts + t1, sizeof(u64), hipMemcpyDeviceToHost,
                                 stream));
            sync();
            const u64 j0 = std::min(t0 * tile_out, n + total) - h_small[2];
            const u64 j1 = std::min(t1 * tile_out, n + total) - h_small[3];
            m = j1 - j0;
          }
          st.candidates += m;
          absorb<K>(H, kp<K>(jchunk), m);
        }
        return;
      }
      K* out;
      u64 base = 0;
      if (last) {
        reserve_keep(H.cand, H.n_cand * sizeof(K), (H.n_cand + total) * sizeof(K),
                     chunk_bytes());
        out = kp<K>(H.cand);
        base = H.n_cand;
      } else {
        reserve_grow(tmp[ping], total * sizeof(K));
        out = kp<K>(tmp[ping]);
      }
      if (filtered) {
        h_small[0] = base;
        HIPCK(hipMemcpyAsync(d_cursor, h_small, sizeof(u64), hipMemcpyHostToDevice, stream));
      }
      HIPCK(hl::wide_expand_tiles<K>(cur, n, static_cast<u64*>(join_off.p),
                                     static_cast<u32*>(join_start.p), inner, total, ws, parts, 0,
                                     nt, filtered ? out : out + base, d_cursor, stream, kt()));
      u64 produced = total;
      if (filtered) {
        HIPCK(hipMemcpyAsync(h_small, d_cursor, sizeof(u64), hipMemcpyDeviceToHost, stream));
        sync();
        produced = h_small[0] - base;
      }
      if (last) {
        H.n_cand += produced;
        st.candidates += produced;
      } else {
        cur = kp<K>(tmp[ping]);
        n = produced;
        ping ^= 1;
        if (n == 0) return;
      }
    }
  }

  // Outer tuples one join pass takes: a larger outer joins a slice at a
  // time, which bounds the per-outer-tuple scratch of the probe and scan
  // (16 bytes per tuple) and the intermediate results of multi-atom rules;
  // the slices' outputs are appended like one pass's.
  u64 outer_slice = u64(1) << 28;  // hl_options.outer_slice_log2

  // Evaluates one plan, appending head tuples to the head's candidates.
  template <typename K>
  void run_plan(const Plan& p) {
    Relation& O = rels[p.outer_rel];
    const K* outer = p.outer_delta ? kp<K>(O.delta) : kp<K>(O.full);
    const u64 n = p.outer_delta ? O.n_delta : O.n_full;
    for (u64 o = 0; o < n; o += outer_slice)
      run_plan_on<K>(p, outer + o, std::min(outer_slice, n - o));
  }

  template <typename K>
  void run_plan_on(const Plan& p, const K* cur, u64 n) {
    Relation& H = rels[p.head];
    if (n == 0) return;
    u64* d_cursor = d_small;
    if (p.steps.empty()) {
      JoinSpec js = p.proj;
      js.w = w;
      H.raw_cand += n;
      st.join_outputs += n;
      rule_out[p.rule] += n;
      reserve_keep(H.cand, H.n_cand * sizeof(K), (H.n_cand + n) * sizeof(K));
      const bool filtered = js.fa >= 0 || js.ea >= 0;
      if (filtered) {
        h_small[0] = H.n_cand;
        HIPCK(hipMemcpyAsync(d_cursor, h_small, sizeof(u64), hipMemcpyHostToDevice, stream));
      }
      HIPCK(hl::project<K>(cur, n, js, kp<K>(H.cand) + (filtered ? 0 : H.n_cand), d_cursor,
                           stream));
      if (filtered) {
        HIPCK(hipMemcpyAsync(h_small, d_cursor, sizeof(u64), hipMemcpyDeviceToHost, stream));
        sync();
        st.candidates += h_small[0] - H.n_cand;
        H.n_cand = h_small[0];
      } else {
        H.n_cand += n;
        st.candidates += n;
      }
      return;
    }
    if ((flags & HL_FLAG_NESTED_JOINS) && p.steps.size() == 2 && run_nested<K>(p, cur, n)) return;
    int ping = 0;
    for (size_t q = 0; q < p.steps.size(); ++q) {
      const Step& s = p.steps[q];
      Relation& I = rels[s.inner_rel];
      Index& ix = I.idx[s.inner_col];
      if (ix.n == 0 || (learned() ? !ix.lm_ok : ix.cap == 0)) return;
      const K* inner = s.inner_col == 0 ? kp<K>(I.full) : kp<K>(ix.keys);
      // an inner kept as two levels: its tail run is probed through the
      // tail's own index, and the expand covers both runs of every outer
      // tuple (entries n + i are outer tuple i's runs in the tail)
      Index& tx = I.tidx[s.inner_col];
      const bool two = I.n_tail > 0 && tx.n > 0 && levels_ok(I);
      const K* inner2 = two ? (s.inner_col == 0 ? kp<K>(I.fz_tail[0]) : kp<K>(tx.keys)) : nullptr;
      JoinSpec js = s.js;
      js.w = w;
      if (n >= (u64(1) << 32) || (two && 2 * n >= (u64(1) << 32)))
        fail(HL_E_UNSUPPORTED, "join outer side of 2^32 or more probes");
      const bool last = q + 1 == p.steps.size();
      js.dd = (last && H.dedup && (flags & HL_FLAG_JOIN_DEDUP)) ? 1 : 0;
      if (js.dd) {
        // Group the outer by the column its outputs carry, so that repeats
        // of one output come from neighbouring outer tuples and fall in one
        // tile: a stable sort on that column's bits.  A delta or full outer
        // is already sorted by column 0.
        const int c = 1 - js.outer_col;
        const int g = (js.src0 == c || js.src1 == c) ? c : js.outer_col;
        if (!(g == 0 && q == 0)) {
          reserve_grow(grp[0], n * sizeof(K));
          reserve_grow(grp[1], n * sizeof(K));
          HIPCK(hipMemcpyAsync(grp[0].p, cur, n * sizeof(K), hipMemcpyDeviceToDevice, stream));
          reserve(ws, hl::sort_workspace_bytes(n), hl::sort_workspace_bytes(n) * 2);
          K* grouped = nullptr;
          HIPCK(hl::radix_sort_bits<K>(kp<K>(grp[0]), kp<K>(grp[1]), n, g == 0 ? w : 0,
                                       g == 0 ? 2 * w : w, ws.p, stream, &grouped, kt(),
                                       sort_items));
          cur = grouped;
        }
      }
      const u64 ne = two ? 2 * n : n;  // probe entries
      reserve_grow(join_start, ne * sizeof(u32));
      reserve_grow(join_len, ne * sizeof(u32));
      reserve_grow(join_off, ne * sizeof(u64));
      for (int level = 0; level < (two ? 2 : 1); ++level) {
        Index& lx = level ? tx : ix;
        u32* st_p = static_cast<u32*>(join_start.p) + (level ? n : 0);
        u32* ln_p = static_cast<u32*>(join_len.p) + (level ? n : 0);
        if (learned())
          HIPCK(hl::join_probe_learned<K>(cur, n, js, lx.view<K>(), st_p, ln_p, stream, kt()));
        else
          HIPCK(hl::join_probe<K>(cur, n, js, static_cast<const Slot*>(lx.table.p), lx.cap, st_p,
                                  ln_p, stream, kt()));
      }
      reserve(ws, hl::scan_workspace_bytes(ne), hl::scan_workspace_bytes(ne) * 2);
      HIPCK(hl::scan_u32_u64(static_cast<u32*>(join_len.p), ne, static_cast<u64*>(join_off.p),
                             d_small + 1, ws.p, stream));
      HIPCK(hipMemcpyAsync(h_small + 1, d_small + 1, sizeof(u64), hipMemcpyDeviceToHost, stream));
      sync();
      const u64 total = h_small[1];
      if (total == 0) return;
      (last ? rule_out : rule_mid)[p.rule] += total;
      if (last) {
        H.raw_cand += total;
        st.join_outputs += total;
      }
      const u64 cap = chunk_keys();
      if (last && total > cap) {
        // One join's outputs exceed one sort: expand a range of tiles at a
        // time (at most `cap` outputs) and absorb each range into the head
        // relation's pending delta, so memory stays bounded by the range.
        const u64 nt = hl::join_tiles(ne, total, join_items);
        reserve_grow(join_parts, hl::join_parts(ne, total, join_items) * sizeof(u64));
        u64* parts = static_cast<u64*>(join_parts.p);
        HIPCK(hl::join_partition(static_cast<u64*>(join_off.p), ne, total, parts, stream,
                                 join_items));
        const u64 tile_out = hl::join_tile_outputs(join_items);
        const u64 per = std::max<u64>(1, cap / tile_out);
        reserve(jchunk, per * tile_out * sizeof(K), per * tile_out * sizeof(K));
        const bool filt = js.fa >= 0 || js.ea >= 0 || js.dd;
        for (u64 t0 = 0; t0 < nt; t0 += per) {
          const u64 tiles = std::min(per, nt - t0);
          if (filt) {
            h_small[0] = 0;
            HIPCK(hipMemcpyAsync(d_cursor, h_small, sizeof(u64), hipMemcpyHostToDevice, stream));
          }
          HIPCK(hl::join_expand_tiles<K>(cur, ne, static_cast<u64*>(join_off.p),
                                         static_cast<u32*>(join_start.p), inner, total, js, parts,
                                         t0, tiles, kp<K>(jchunk), d_cursor, stream, kt(),
                                         join_items, inner2, two ? n : ne));
          u64 m;
          if (filt) {
            HIPCK(hipMemcpyAsync(h_small, d_cursor, sizeof(u64), hipMemcpyDeviceToHost, stream));
            sync();
            m = h_small[0];
          } else {
            // outputs of tiles [t0, t1): j(t1) - j(t0), j(t) = min(t * tile, n + total) - parts[t]
            const u64 t1 = t0 + tiles;
            HIPCK(hipMemcpyAsync(h_small + 2, parts + t0, sizeof(u64), hipMemcpyDeviceToHost,
                                 stream));
            HIPCK(hipMemcpyAsync(h_small + 3, parts + t1, sizeof(u64), hipMemcpyDeviceToHost,
                                 stream));
            sync();
            const u64 j0 = std::min(t0 * tile_out, ne + total) - h_small[2];
            const u64 j1 = std::min(t1 * tile_out, ne + total) - h_small[3];
            m = j1 - j0;
          }
          st.candidates += m;
          absorb<K>(H, kp<K>(jchunk), m);
        }
        return;
      }
      const bool filtered = js.fa >= 0 || js.ea >= 0 || js.dd;
      K* out;
      u64 base = 0;
      if (last) {
        reserve_keep(H.cand, H.n_cand * sizeof(K), (H.n_cand + total) * sizeof(K),
                     chunk_bytes());
        out = kp<K>(H.cand);
        base = H.n_cand;
      } else {
        reserve_grow(tmp[ping], total * sizeof(K));
        out = kp<K>(tmp[ping]);
      }
      if (filtered) {
        h_small[0] = base;
        HIPCK(hipMemcpyAsync(d_cursor, h_small, sizeof(u64), hipMemcpyHostToDevice, stream));
      }
      reserve_grow(join_parts, hl::join_parts(ne, total, join_items) * sizeof(u64));
      HIPCK(hl::join_expand<K>(cur, ne, static_cast<u64*>(join_off.p),
                               static_cast<u32*>(join_start.p), inner, total, js,
                               static_cast<u64*>(join_parts.p), filtered ? out : out + base,
                               d_cursor, stream, kt(), join_items, inner2, two ? n : ne));
      u64 produced = total;
      if (filtered) {
        HIPCK(hipMemcpyAsync(h_small, d_cursor, sizeof(u64), hipMemcpyDeviceToHost, stream));
        sync();
        produced = h_small[0] - base;
      }
      if (last) {
        H.n_cand += produced;
        st.candidates += produced;
      } else {
        cur = kp<K>(tmp[ping]);
        n = produced;
        ping ^= 1;
        if (n == 0) return;
      }
    }
  }

  // A two-join body evaluated by nested loops (HL_FLAG_NESTED_JOINS, the
  // paper's nested joins of Section 5.2, kept as an ablation of the
  // materialised chain): one thread per outer tuple, a counting pass, a
  // scan and a writing pass.  Returns false when the outputs exceed one
  // sort chunk (the materialised chain then runs instead).
  template <typename K>
  bool run_nested(const Plan& p, const K* cur, u64 n) {
    for (const Step& s : p.steps)
      if (rels[s.inner_rel].n_tail > 0 && levels_ok(rels[s.inner_rel]))
        return false;  // an inner kept as two levels: the materialised chain
    Relation& H = rels[p.head];
    hl::NestedJoin<K> nj{};
    for (int q = 0; q < 2; ++q) {
      const Step& s = p.steps[q];
      Relation& I = rels[s.inner_rel];
      Index& ix = I.idx[s.inner_col];
      if (ix.n == 0 || (learned() ? !ix.lm_ok : ix.cap == 0)) return true;  // nothing joins
      nj.inner[q] = s.inner_col == 0 ? kp<K>(I.full) : kp<K>(ix.keys);
      if (learned()) {
        nj.lv[q] = ix.view<K>();
      } else {
        nj.table[q] = static_cast<const Slot*>(ix.table.p);
        nj.cap[q] = ix.cap;
      }
      nj.js[q] = s.js;
      nj.js[q].w = w;
      nj.js[q].dd = 0;
    }
    if (n >= (u64(1) << 32)) fail(HL_E_UNSUPPORTED, "join outer side of 2^32 or more tuples");
    reserve_grow(join_len, n * sizeof(u32));
    reserve_grow(join_off, n * sizeof(u64));
    reserve(ws, hl::scan_workspace_bytes(n), hl::scan_workspace_bytes(n) * 2);
    u32* too_many = reinterpret_cast<u32*>(d_small + 2);
    HIPCK(hl::fill_zero(d_small + 2, sizeof(u64), stream));
    HIPCK(hl::join_nested<K>(cur, n, nj, static_cast<u32*>(join_len.p),
                             static_cast<u64*>(join_off.p), d_small + 1, too_many, ws.p, nullptr,
                             stream));
    HIPCK(hipMemcpyAsync(h_small + 1, d_small + 1, 2 * sizeof(u64), hipMemcpyDeviceToHost,
                         stream));
    sync();
    if (u32(h_small[2]) != 0)
      fail(HL_E_UNSUPPORTED, "nested join: an outer tuple with 2^32 or more outputs");
    const u64 total = h_small[1];
    if (total > chunk_keys()) return false;
    if (total == 0) return true;
    // the nested form counts kept outputs only: they are its join outputs
    H.raw_cand += total;
    rule_out[p.rule] += total;
    st.join_outputs += total;
    reserve_keep(H.cand, H.n_cand * sizeof(K), (H.n_cand + total) * sizeof(K),
                     chunk_bytes());
    HIPCK(hl::join_nested<K>(cur, n, nj, nullptr, static_cast<u64*>(join_off.p), nullptr, nullptr,
                             nullptr, kp<K>(H.cand) + H.n_cand, stream));
    H.n_cand += total;
    st.candidates += total;
    return true;
  }

  // Model of R's full relation for the set difference of n_cand sorted
  // candidates, if it has a current one.  A relation that no join probes
  // gets one fitted here when its candidates are spread thinly over a
  // large full (at least 8 keys of full per candidate), the relation's
  // last difference searched a quarter or more of its tiles in global
  // memory (candidates grouped by their first column keep slices short
  // however large full is), and full is being kept stable by a tail run:
  // the model then lasts until the tail is folded in, and each search
  // starts from the model's window instead of the whole slice.  A full
  // merged anew every iteration would need a fit per difference, which the
  // searches do not repay.
  template <typename K>
  bool diff_model(Relation& R, u64 n_cand, hl::LearnedView<K>* mv) {
    if (!learned() || R.n_full == 0) return false;
    Index& ix = R.idx[0];
    bool use = ix.lm_ok && ix.lm_keys == R.full.p && ix.lm_n == R.n_full;
    if (!use && !ix.used && tail_ok(R) && R.n_full * sizeof(K) >= tail_min_bytes &&
        R.n_full >= 8 * n_cand && R.lockstep_share >= 0.25 && R.n_tail > 0) {
      const int caller = marks.empty() ? -1 : marks.back().first;
      mark(HL_PHASE_INDEX);
      fit_model<K>(R, 0);
      mark(caller);
      use = ix.lm_ok;
    }
    if (use) *mv = ix.view<K>();
    return use;
  }

  // Absorbs m new tuples (unsorted, at `keys`, which is overwritten) into
  // R's pending delta: they are sorted, cut down to the distinct ones that
  // are neither in full nor already pending, and merged in (the pieces are
  // disjoint, so the merge needs no dedup).  One synchronisation.
  // Its sort, difference and merge are charged to those phases; the
  // caller's phase (the join, when a join's outputs are absorbed range by
  // range) resumes afterwards.
  template <typename K>
  void absorb(Relation& R, K* keys, u64 m) {
    if (m == 0) return;
    const int caller = marks.empty() ? -1 : marks.back().first;
    struct Resume {
      hl_engine* e;
      int ph;
      ~Resume() {
        if (e->marks.empty() || e->marks.back().first != ph) {
          try {
            e->mark(ph);
          } catch (...) {
          }
        }
      }
    } resume{this, caller};
    const int bits = kbits(R);
    reserve_chunk(alt, m * sizeof(K));
    reserve(ws, hl::sort_workspace_bytes(m), hl::sort_workspace_bytes(m) * 2);
    K* sorted = nullptr;
    mark(HL_PHASE_SORT);
    HIPCK(hl::radix_sort<K>(keys, kp<K>(alt), m, bits, ws.p, stream, &sorted, kt(), sort_items));
    K* other = sorted == keys ? kp<K>(alt) : keys;
    mark(HL_PHASE_DIFF);
    reserve(ws, hl::unique_diff_workspace_bytes(m), hl::unique_diff_workspace_bytes(m) * 2);
    u64* dc = d_small + kChunkSlots;  // scratch counts (not the per-relation slots)
    u64* hc = h_small + kChunkSlots;
    hl::LearnedView<K> mv{};
    const bool use_model = diff_model<K>(R, m, &mv);
    // the tail run beside full, if any, is tested in the same pass
    HIPCK(hl::fill_zero(dc + 2, sizeof(u64), stream));
    HIPCK(hl::unique_diff<K>(sorted, m, kp<K>(R.full), R.n_full, other, sorted, dc, ws.p, stream,
                             kt(), use_model ? &mv : nullptr,
                             R.n_tail ? kp<K>(R.fz_tail[0]) : nullptr, R.n_tail, diff_items,
                             dc + 2));
    HIPCK(hipMemcpyAsync(hc, dc, 3 * sizeof(u64), hipMemcpyDeviceToHost, stream));
    sync();
    R.lockstep_share = double(hc[2]) / double(diff_tiles(m));
    u64 d = hc[0];
    R.pend_uniq += hc[1];
    const u64 p = R.n_pend;
    if (p > 0 && d > 0) {
      HIPCK(hl::unique_diff<K>(sorted, d, kp<K>(R.pend[0]), p, other, sorted, dc, ws.p, stream,
                               kt(), nullptr, nullptr, 0, diff_items));
      HIPCK(hipMemcpyAsync(hc, dc, sizeof(u64), hipMemcpyDeviceToHost, stream));
      sync();
      d = hc[0];
    }
    if (d == 0) return;
    mark(HL_PHASE_MERGE);
    if (p == 0) {
      reserve(R.pend[0], d * sizeof(K), d * sizeof(K) * 3 / 2);
      HIPCK(hipMemcpyAsync(R.pend[0].p, sorted, d * sizeof(K), hipMemcpyDeviceToDevice, stream));
    } else {
      reserve(R.pend[1], (p + d) * sizeof(K), (p + d) * sizeof(K) * 3 / 2);
      reserve(ws, hl::merge_workspace_bytes(p, d), hl::merge_workspace_bytes(p, d) * 2);
      HIPCK(hl::merge<K>(kp<K>(R.pend[0]), p, sorted, d, kp<K>(R.pend[1]), ws.p, stream, kt()));
      std::swap(R.pend[0], R.pend[1]);
    }
    R.n_pend = p + d;
  }

  // Delta of a relation that has pending tuples or whose new tuples exceed
  // one sort chunk (chunk_keys()): the candidates are absorbed chunk by
  // chunk and the pending set becomes delta.  Returns (|delta|, sum over
  // chunks of their distinct tuples).
  template <typename K>
  std::pair<u64, u64> chunked_delta(Relation& R) {
    const u64 kChunk = chunk_keys();
    for (u64 c = 0; c < R.n_cand; c += kChunk)
      absorb<K>(R, kp<K>(R.cand) + c, std::min(kChunk, R.n_cand - c));
    std::swap(R.delta, R.pend[0]);
    const std::pair<u64, u64> r{R.n_pend, R.pend_uniq};
    R.n_pend = R.pend_uniq = 0;
    return r;
  }

  // Sort + unique + subtraction of full for every IDB relation, then the
  // merges and index refreshes.  Returns the total delta size.
  template <typename K>
  u64 close_iteration() {
    std::vector<int> idbs;
    for (int k = 0; k < int(rels.size()); ++k)
      if (!rels[k].edb) idbs.push_back(k);
    if (2 * idbs.size() > kChunkSlots) fail(HL_E_UNSUPPORTED, "too many relations");
    // the deltas become the new outers: free their old contents
    mark(HL_PHASE_SORT);
    std::vector<std::pair<size_t, std::pair<u64, u64>>> chunked;
    for (size_t q = 0; q < idbs.size(); ++q) {
      Relation& R = rels[idbs[q]];
      R.n_delta = 0;
      if (R.n_cand == 0 && R.n_pend == 0) {
        HIPCK(hl::fill_zero(d_small + 2 * q, 2 * sizeof(u64), stream));
        continue;
      }
      if (R.n_pend > 0 || R.n_cand > chunk_keys()) {
        chunked.push_back({q, chunked_delta<K>(R)});
        HIPCK(hl::fill_zero(d_small + 2 * q, 2 * sizeof(u64), stream));
        continue;
      }
      reserve_chunk(alt, R.n_cand * sizeof(K));
      reserve(ws, hl::sort_workspace_bytes(R.n_cand), hl::sort_workspace_bytes(R.n_cand) * 2);
      K* sorted = nullptr;
      mark(HL_PHASE_SORT);
      HIPCK(hl::radix_sort<K>(kp<K>(R.cand), kp<K>(alt), R.n_cand, kbits(R), ws.p, stream,
                              &sorted, kt(), sort_items));
      Buf& sbuf = (sorted == kp<K>(R.cand)) ? R.cand : alt;
      Buf& obuf = (sorted == kp<K>(R.cand)) ? alt : R.cand;
      reserve(ws, hl::unique_diff_workspace_bytes(R.n_cand),
              hl::unique_diff_workspace_bytes(R.n_cand) * 2);
      mark(HL_PHASE_DIFF);
      hl::LearnedView<K> mv{};
      const bool use_model = diff_model<K>(R, R.n_cand, &mv);
      // a tail run beside full is tested in the same pass; the survivors
      // stay in obuf until their count is known, then go to delta (which
      // is sized by that count: handing delta the candidates' block would
      // make both roles candidate-sized)
      u64* d_lock = d_small + kChunkSlots + 2;
      HIPCK(hl::fill_zero(d_lock, sizeof(u64), stream));
      HIPCK(hl::unique_diff<K>(kp<K>(sbuf), R.n_cand, kp<K>(R.full), R.n_full, kp<K>(obuf),
                               static_cast<K*>(nullptr), d_small + 2 * q, ws.p, stream, kt(),
                               use_model ? &mv : nullptr,
                               R.n_tail ? kp<K>(R.fz_tail[0]) : nullptr, R.n_tail, diff_items,
                               d_lock));
      HIPCK(hipMemcpyAsync(h_small + 2 * q, d_small + 2 * q, sizeof(u64), hipMemcpyDeviceToHost,
                           stream));
      HIPCK(hipMemcpyAsync(h_small + kChunkSlots + 2, d_lock, sizeof(u64), hipMemcpyDeviceToHost,
                           stream));
      sync();
      R.lockstep_share = double(h_small[kChunkSlots + 2]) / double(diff_tiles(R.n_cand));
      const u64 D = h_small[2 * q];
      if (D > 0) {
        reserve_grow(R.delta, D * sizeof(K));
        HIPCK(hl::unique_diff_gather<K>(kp<K>(obuf), R.n_cand, R.n_full, ws.p, kp<K>(R.delta),
                                        stream, diff_items));
      }
    }
    HIPCK(hipMemcpyAsync(h_small, d_small, 2 * idbs.size() * sizeof(u64), hipMemcpyDeviceToHost,
                         stream));
    mark(-1);
    sync();
    collect();
    for (auto& c : chunked) {
      h_small[2 * c.first] = c.second.first;
      h_small[2 * c.first + 1] = c.second.second;
    }
    u64 total = 0;
    // grown: full took the delta (indexes refreshed with it); folded: full
    // took a two-level relation's tail, whose indexes already hold the
    // delta; tail_grown: only the tail of a two-level relation grew
    std::vector<int> grown, folded, tail_grown;
    mark(HL_PHASE_MERGE);
    for (size_t q = 0; q < idbs.size(); ++q) {
      Relation& R = rels[idbs[q]];
      const u64 D = h_small[2 * q], U = h_small[2 * q + 1];
      if (R.raw_cand > 0) R.dedup = double(R.raw_cand) >= 1.5 * double(U);
      R.raw_cand = 0;
      R.n_delta = D;
      R.delta_counts.push_back(D);
      R.new_counts.push_back(U);
      R.n_cand = 0;
      total += D;
      if (D == 0) continue;
      const u64 F = R.n_full;
      if (levels_ok(R) && F * sizeof(K) >= tail_min_bytes) {
        // a relation probed as a join inner, kept as two levels: a small
        // delta goes into the tail run and the tail's indexes, so full and
        // its indexes stay as they are; a delta that would make the tail
        // larger than an eighth of full folds the tail into full, whose
        // indexes are then refreshed
        delta_into_tail<K>(R);
        if (R.n_tail * 8 <= F) {
          tail_grown.push_back(idbs[q]);
        } else {
          fold_inner_tail<K>(R);
          folded.push_back(idbs[q]);
        }
        continue;
      }
      if (R.n_tail > 0 && levels_ok(R)) {
        // full shrank below the threshold (a new run): fold first
        fold_inner_tail<K>(R);
      }
      if (tail_ok(R) && F * sizeof(K) >= tail_min_bytes && (R.n_tail + D) * 8 <= F) {
        // small delta against a large full: merge it into the tail run only
        const u64 T = R.n_tail;
        if (T == 0) {
          reserve(R.fz_tail[0], D * sizeof(K), u64(ebm_k * double(D) * sizeof(K)));
          HIPCK(hipMemcpyAsync(R.fz_tail[0].p, R.delta.p, D * sizeof(K), hipMemcpyDeviceToDevice,
                               stream));
        } else {
          reserve(R.fz_tail[1], (T + D) * sizeof(K), u64((double(T) + ebm_k * double(D)) * sizeof(K)));
          reserve(ws, hl::merge_workspace_bytes(T, D), hl::merge_workspace_bytes(T, D) * 2);
          HIPCK(hl::merge<K>(kp<K>(R.fz_tail[0]), T, kp<K>(R.delta), D, kp<K>(R.fz_tail[1]), ws.p,
                             stream, kt()));
          std::swap(R.fz_tail[0], R.fz_tail[1]);
        }
        R.n_tail = T + D;
        grown.push_back(idbs[q]);
        continue;
      }
      if (R.n_tail > 0) {
        // the tail takes the delta, then folds into full
        const u64 T = R.n_tail;
        reserve(R.fz_tail[1], (T + D) * sizeof(K), u64((double(T) + ebm_k * double(D)) * sizeof(K)));
        reserve(ws, hl::merge_workspace_bytes(T, D), hl::merge_workspace_bytes(T, D) * 2);
        HIPCK(hl::merge<K>(kp<K>(R.fz_tail[0]), T, kp<K>(R.delta), D, kp<K>(R.fz_tail[1]), ws.p,
                           stream, kt()));
        std::swap(R.fz_tail[0], R.fz_tail[1]);
        R.n_tail = T + D;
        flush_tail<K>(R);
        grown.push_back(idbs[q]);
        continue;
      }
      if (F == 0) {
        reserve(R.full, D * sizeof(K), u64(ebm_k * double(D) * sizeof(K)));
        HIPCK(hipMemcpyAsync(R.full.p, R.delta.p, D * sizeof(K), hipMemcpyDeviceToDevice, stream));
      } else {
        reserve(R.full_spare, (F + D) * sizeof(K), u64((double(F) + ebm_k * double(D)) * sizeof(K)));
        reserve(ws, hl::merge_workspace_bytes(F, D), hl::merge_workspace_bytes(F, D) * 2);
        HIPCK(hl::merge<K>(kp<K>(R.full), F, kp<K>(R.delta), D, kp<K>(R.full_spare), ws.p, stream,
                           kt()));
        std::swap(R.full, R.full_spare);
      }
      R.n_full = F + D;
      R.idx[0].n = R.n_full;
      grown.push_back(idbs[q]);
    }
    mark(HL_PHASE_INDEX);
    if (wide) {
      for (int r : grown)
        for (Index& ix : rels[r].widx)
          update_wide<K>(rels[r], ix, kp<K>(rels[r].delta), rels[r].n_delta, false);
      refresh_wide<K>(grown);
    } else {
      for (int r : grown) update_swapped<K>(rels[r], kp<K>(rels[r].delta), rels[r].n_delta, false);
      grown.insert(grown.end(), folded.begin(), folded.end());
      refresh_indexes<K>(grown);
      refresh_tail_indexes<K>(tail_grown);
    }
    mark(-1);
    return total;
  }

  // ------------------------------------------------- fused iterations

  bool fused_on() const {
    return (flags & (HL_FLAG_FUSED | HL_FLAG_HIP_GRAPH)) && !(flags & HL_FLAG_NO_EBM) && fz_plans;
  }

  // LDS capacities for key type K: for a joining workgroup the largest
  // power-of-two candidate buffer (and half of it for a first join's
  // result) that fits the device's LDS per workgroup; for the finishing
  // workgroup, which holds only keys, the largest power of two that fits.
  template <typename K>
  void fused_setup() {
    if (fz_key_bytes == int(sizeof(K))) return;
    int lds = 0;
    HIPCK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    const u64 avail = u64(lds) > 1024 ? u64(lds) - 1024 : 0;  // static LDS of the kernel
    u32 c = 0;
    for (u32 t = 2; t <= 16384; t <<= 1)
      if (hl::fused_lds_bytes<K>(t, t / 2) <= avail) c = t;
    if (c < 1024) fail(HL_E_UNSUPPORTED, "fused iterations need more LDS per workgroup");
    u32 b = c;
    while (b < 32768 && u64(2 * b) * sizeof(K) <= avail) b *= 2;
    if (fused_capacity) {
      if (fused_capacity > b)
        fail(HL_E_UNSUPPORTED, "fused_capacity exceeds the LDS of one workgroup");
      b = fused_capacity;
      c = std::min(c, b);
    }
    HIPCK(hl::fused_prepare<K>(c, c / 2, b));
    fz_cap_c = c;
    fz_cap_t = c / 2;
    fz_cap_b = b;
    fz_key_bytes = int(sizeof(K));
  }

  // A fused iteration's tail run next to a full below kTailMinFullBytes
  // holds at most this many keys (2 MB of 64-bit keys, so its membership
  // searches stay in L2); a longer one is folded into full first.
  static constexpr u64 kTailKeys = u64(1) << 18;
  // On the multi-kernel path a relation keeps a tail run once its full
  // holds this many bytes and the tail stays within an eighth of it.  The
  // set difference searches the tail for the keys that survive full, in
  // the same pass; below this size rewriting full costs less than those
  // searches.
  static constexpr u64 kTailMinFullBytes = u64(64) << 20;
  u64 tail_min_bytes = kTailMinFullBytes;  // hl_options.tail_min_bytes
  // Fused iterations fold a long tail into a full below this size (one
  // merge of well under a millisecond) rather than merge into it each time.
  static constexpr u64 kFoldLimitBytes = u64(1) << 30;

  // Whether relation R, probed as a join inner, may be kept as two levels
  // (full with its indexes, plus a tail run with indexes of its own).
  bool levels_ok(const Relation& R) const {
    return !R.edb && !wide && (R.idx[0].used || R.idx[1].used) &&
           !(flags & (HL_FLAG_NO_EBM | HL_FLAG_NO_LEVELS));
  }

  // Merges R's delta into its tail run (and the tail's column-swapped copy
  // when column 1 is probed).
  template <typename K>
  void delta_into_tail(Relation& R) {
    const u64 T = R.n_tail, D = R.n_delta;
    if (T == 0) {
      reserve(R.fz_tail[0], D * sizeof(K), u64(ebm_k * double(D) * sizeof(K)));
      HIPCK(hipMemcpyAsync(R.fz_tail[0].p, R.delta.p, D * sizeof(K), hipMemcpyDeviceToDevice,
                           stream));
    } else {
      reserve(R.fz_tail[1], (T + D) * sizeof(K), u64((double(T) + ebm_k * double(D)) * sizeof(K)));
      reserve(ws, hl::merge_workspace_bytes(T, D), hl::merge_workspace_bytes(T, D) * 2);
      HIPCK(hl::merge<K>(kp<K>(R.fz_tail[0]), T, kp<K>(R.delta), D, kp<K>(R.fz_tail[1]), ws.p,
                         stream, kt()));
      std::swap(R.fz_tail[0], R.fz_tail[1]);
    }
    R.n_tail = T + D;
    R.tidx[0].n = R.n_tail;
    if (R.idx[1].used) {
      // the tail's swapped copy takes the swapped, sorted delta
      Index& tx = R.tidx[1];
      reserve_grow(alt, D * sizeof(K));
      reserve_grow(tmp[0], D * sizeof(K));
      HIPCK(hl::swap_cols<K>(kp<K>(R.delta), D, w, kp<K>(tmp[0]), stream));
      reserve(ws, hl::sort_workspace_bytes(D), hl::sort_workspace_bytes(D) * 2);
      K* sorted = nullptr;
      HIPCK(hl::radix_sort<K>(kp<K>(tmp[0]), kp<K>(alt), D, 2 * w, ws.p, stream, &sorted, kt(),
                              sort_items));
      if (tx.n == 0) {
        reserve(tx.keys, D * sizeof(K), u64(ebm_k * double(D) * sizeof(K)));
        HIPCK(hipMemcpyAsync(tx.keys.p, sorted, D * sizeof(K), hipMemcpyDeviceToDevice, stream));
      } else {
        reserve(tx.spare, (tx.n + D) * sizeof(K),
                u64((double(tx.n) + ebm_k * double(D)) * sizeof(K)));
        reserve(ws, hl::merge_workspace_bytes(tx.n, D), hl::merge_workspace_bytes(tx.n, D) * 2);
        HIPCK(hl::merge<K>(kp<K>(tx.keys), tx.n, sorted, D, kp<K>(tx.spare), ws.p, stream, kt()));
        std::swap(tx.keys, tx.spare);
      }
      tx.n += D;
    }
  }

  // Folds the tail of a two-level relation into full, and the tail's
  // swapped copy into full's; full's indexes must be refreshed afterwards.
  template <typename K>
  void fold_inner_tail(Relation& R) {
    if (R.idx[1].used && R.tidx[1].n > 0) {
      Index& ix = R.idx[1];
      Index& tx = R.tidx[1];
      const u64 total = ix.n + tx.n;
      reserve(ix.spare, total * sizeof(K), u64((double(ix.n) + ebm_k * double(tx.n)) * sizeof(K)));
      reserve(ws, hl::merge_workspace_bytes(ix.n, tx.n), hl::merge_workspace_bytes(ix.n, tx.n) * 2);
      HIPCK(hl::merge<K>(kp<K>(ix.keys), ix.n, kp<K>(tx.keys), tx.n, kp<K>(ix.spare), ws.p, stream,
                         kt()));
      std::swap(ix.keys, ix.spare);
      ix.n = total;
    }
    flush_tail<K>(R);
  }

  // Hash tables (one synchronisation for the run counts of all of them) or
  // learned models of the tail indexes of the listed two-level relations.
  template <typename K>
  void refresh_tail_indexes(const std::vector<int>& which) {
    std::vector<std::pair<int, int>> todo;
    for (int r : which)
      for (int c = 0; c < 2; ++c)
        if (rels[r].idx[c].used) todo.push_back({r, c});
    if (todo.empty()) return;
    auto keys_of = [&](Relation& R, int c) {
      return c == 0 ? kp<K>(R.fz_tail[0]) : kp<K>(R.tidx[1].keys);
    };
    if (learned()) {
      for (auto& rc : todo) {
        Relation& R = rels[rc.first];
        fit_index_model<K>(R, R.tidx[rc.second], keys_of(R, rc.second));
      }
      return;
    }
    if (todo.size() > kChunkSlots) fail(HL_E_UNSUPPORTED, "too many indexes");
    for (size_t q = 0; q < todo.size(); ++q) {
      Relation& R = rels[todo[q].first];
      HIPCK(hl::hisa_count_runs<K>(keys_of(R, todo[q].second), R.tidx[todo[q].second].n, w,
                                   d_small + q, stream));
    }
    HIPCK(hipMemcpyAsync(h_small, d_small, todo.size() * sizeof(u64), hipMemcpyDeviceToHost,
                         stream));
    sync();
    for (size_t q = 0; q < todo.size(); ++q) {
      Relation& R = rels[todo[q].first];
      Index& tx = R.tidx[todo[q].second];
      const u64 runs = h_small[q];
      tx.runs = runs;
      u64 cap = u64(std::ceil(double(runs) / load_factor));
      cap = std::max(cap, runs + 1);
      cap = std::max<u64>(cap, 16);
      reserve(tx.table, cap * sizeof(Slot), cap * sizeof(Slot) * 2);
      tx.cap = cap;
      HIPCK(hl::fill_zero(tx.table.p, cap * sizeof(Slot), stream));
      HIPCK(hl::hisa_build<K>(keys_of(R, todo[q].second), tx.n, w,
                              static_cast<Slot*>(tx.table.p), cap, stream, kt()));
    }
  }

  // Folds R's tail run into its full relation (one merge).
  template <typename K>
  void flush_tail(Relation& R) {
    if (R.n_tail == 0) return;
    const u64 F = R.n_full, T = R.n_tail;
    if (F == 0) {
      reserve(R.full, T * sizeof(K), u64(ebm_k * double(T) * sizeof(K)));
      HIPCK(hipMemcpyAsync(R.full.p, R.fz_tail[0].p, T * sizeof(K), hipMemcpyDeviceToDevice,
                           stream));
    } else {
      reserve(R.full_spare, (F + T) * sizeof(K), u64((double(F) + ebm_k * double(T)) * sizeof(K)));
      reserve(ws, hl::merge_workspace_bytes(F, T), hl::merge_workspace_bytes(F, T) * 2);
      HIPCK(hl::merge<K>(kp<K>(R.full), F, kp<K>(R.fz_tail[0]), T, kp<K>(R.full_spare), ws.p,
                         stream, kt()));
      std::swap(R.full, R.full_spare);
    }
    R.n_full = F + T;
    R.idx[0].n = R.n_full;
    R.n_tail = 0;
    for (Index& tx : R.tidx) {
      tx.n = tx.cap = 0;
      tx.lm_ok = false;
    }
    fz_live = false;  // the fused path's device counts describe the old split
  }

  // Folds every tail run into its full relation.
  template <typename K>
  void flush_tails() {
    bool any = false;
    for (Relation& R : rels) {
      if (R.edb || R.n_tail == 0) continue;
      if (!any) mark(HL_PHASE_MERGE);
      any = true;
      flush_tail<K>(R);
    }
    if (any) mark(-1);
  }

  // Whether R may keep a tail run on the multi-kernel path: no join probes
  // it (its indexes would have to cover the tail), and eager buffers are on.
  bool tail_ok(const Relation& R) const {
    return !R.edb && !R.idx[0].used && !R.idx[1].used && R.widx.empty() &&
           !(flags & HL_FLAG_NO_EBM);
  }

  void drop_graphs() {
    for (auto& g : fz_graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    fz_graphs.clear();
  }

  // Whether the next iteration should try the fused path: the last
  // iteration's join outputs per outer tuple predict the candidates.
  bool fused_next(u64 sum_delta) const {
    if (!fused_on() || sum_delta == 0 || sum_delta >= fz_fail_at) return false;
    const double rate = last_in ? double(last_out) / double(last_in) : 1.0;
    return double(sum_delta) * std::max(rate, 1.0) <= 0.9 * double(fz_cap_b);
  }

  // One iteration of the recursive stratum as a fused launch plus
  // device-sized merges.  Returns false, with the state unchanged, when the
  // candidates did not fit (the caller then runs the multi-kernel path);
  // otherwise *total receives the total delta size.
  template <typename K>
  bool fused_iteration(u64* total) {
    mark(HL_PHASE_FUSED);
    fused_setup<K>();
    std::vector<int> idbs, slot(rels.size(), -1);
    for (int k = 0; k < int(rels.size()); ++k)
      if (!rels[k].edb) {
        slot[k] = int(idbs.size());
        idbs.push_back(k);
      }
    const u64 C = fz_cap_b;  // most new tuples one relation gets per iteration
    hl::FusedIteration<K> it{};
    it.nrels = int(idbs.size());
    it.w = w;
    for (const Plan& p : plansR) {
      hl::FusedPlan<K> fp{};
      fp.outer = slot[p.outer_rel];
      fp.head = slot[p.head];
      fp.nsteps = int(p.steps.size());
      bool empty_inner = false;
      if (p.steps.empty()) {
        fp.steps[0].js = p.proj;
        fp.steps[0].js.w = w;
      }
      for (size_t q = 0; q < p.steps.size(); ++q) {
        const Step& s = p.steps[q];
        Relation& I = rels[s.inner_rel];
        Index& ix = I.idx[s.inner_col];
        if (ix.n == 0 || (learned() ? !ix.lm_ok : ix.cap == 0)) empty_inner = true;
        hl::FusedStep<K>& fs = fp.steps[q];
        fs.inner = s.inner_col == 0 ? kp<K>(I.full) : kp<K>(ix.keys);
        if (learned()) fs.lv = ix.view<K>();
        else {
          fs.table = static_cast<const Slot*>(ix.table.p);
          fs.cap = ix.cap;
        }
        fs.js = s.js;
        fs.js.w = w;
        fs.js.dd = 0;
      }
      if (!empty_inner) it.plans[it.nplans++] = fp;  // an empty inner joins nothing
    }
    // The tail may grow by C keys this iteration.  Past kTailKeys it is
    // folded into full first, unless full is so large that folding costs
    // more than merging the longer tail for the rest of the fused
    // iterations (then it is folded once it reaches an eighth of full, as
    // on the multi-kernel path).
    for (int r : idbs) {
      Relation& R = rels[r];
      const bool big = R.n_full * sizeof(K) >= kFoldLimitBytes;
      if (R.n_tail + C > (big ? R.n_full / 8 : kTailKeys)) {
        mark(HL_PHASE_MERGE);
        flush_tail<K>(R);
        mark(-1);
      }
    }
    std::vector<u64> max_out(idbs.size());
    for (size_t r = 0; r < idbs.size(); ++r) {
      Relation& R = rels[idbs[r]];
      reserve(R.fz_next, C * sizeof(K), C * sizeof(K));
      // the merge grid covers 8 more full-capacity deltas, so a captured
      // graph serves several iterations
      max_out[r] = (R.n_tail + C + 8 * C - 1) / (8 * C) * (8 * C);
      // the merge target holds the tail and one more delta (with room for
      // the grid's span, so the pair of buffers settles after two rounds)
      const u64 want = std::max<u64>(kTailKeys, max_out[r]);
      reserve(R.fz_tail[1], (R.n_tail + C) * sizeof(K), want * sizeof(K));
      const u64 parts = (hl::fused_merge_tiles(max_out[r]) + 1) * sizeof(u64);
      reserve(R.fz_parts, parts, (hl::fused_merge_tiles(want) + 1) * sizeof(u64));
      it.delta_in[r] = kp<K>(R.delta);
      it.full[r] = kp<K>(R.full);
      hl::LearnedView<K> mv{};
      if (diff_model<K>(R, C, &mv)) it.full_lm[r] = mv;
      it.tail[r] = kp<K>(R.fz_tail[0]);
      it.delta_out[r] = kp<K>(R.fz_next);
    }
    it.counts = d_fz;
    const u64 scratch = hl::fused_scratch_bytes<K>(fz_cap_c, it.nrels);
    reserve(fz_scratch, scratch, scratch);
    if (!fz_live) {
      for (int k = 0; k < hl::kFusedCountWords; ++k) h_fz[k] = 0;
      for (size_t r = 0; r < idbs.size(); ++r) {
        h_fz[r * hl::kFusedSlots + 0] = rels[idbs[r]].n_delta;
        h_fz[r * hl::kFusedSlots + 1] = rels[idbs[r]].n_full;
        h_fz[r * hl::kFusedSlots + 6] = rels[idbs[r]].n_tail;
      }
      HIPCK(hipMemcpyAsync(d_fz, h_fz, hl::kFusedCountWords * sizeof(u64), hipMemcpyHostToDevice,
                           stream));
    }
    auto enqueue = [&] {
      HIPCK(hl::fused_iteration<K>(it, fz_cap_c, fz_cap_t, fz_cap_b, fz_scratch.p, stream));
      for (size_t r = 0; r < idbs.size(); ++r) {
        Relation& R = rels[idbs[r]];
        HIPCK(hl::fused_merge<K>(kp<K>(R.fz_tail[0]), kp<K>(R.fz_next), d_fz, int(r), max_out[r],
                                 static_cast<u64*>(R.fz_parts.p), kp<K>(R.fz_tail[1]), stream));
      }
      HIPCK(hl::fused_advance(d_fz, it.nrels, stream));
      HIPCK(hipMemcpyAsync(h_fz, d_fz, hl::kFusedCountWords * sizeof(u64), hipMemcpyDeviceToHost,
                           stream));
    };
    mark(HL_PHASE_FUSED);
    if (flags & HL_FLAG_HIP_GRAPH) {
      // the graph is keyed by everything its launches capture: the
      // iteration's description, the merge targets and grids
      std::vector<unsigned char> key(sizeof(it));
      std::memcpy(key.data(), &it, sizeof(it));
      auto add = [&](const void* p, size_t n) {
        const unsigned char* b = static_cast<const unsigned char*>(p);
        key.insert(key.end(), b, b + n);
      };
      for (size_t r = 0; r < idbs.size(); ++r) {
        const void* ptrs[2] = {rels[idbs[r]].fz_tail[1].p, rels[idbs[r]].fz_parts.p};
        add(ptrs, sizeof(ptrs));
        add(&max_out[r], sizeof(u64));
      }
      add(&fz_cap_c, sizeof(fz_cap_c));
      add(&fz_cap_b, sizeof(fz_cap_b));
      add(&fz_scratch.p, sizeof(fz_scratch.p));
      FzGraph* g = nullptr;
      for (auto& c : fz_graphs)
        if (c.key == key) g = &c;
      if (!g) {
        if (fz_graphs.size() >= 4) {
          (void)hipGraphExecDestroy(fz_graphs.front().exec);
          fz_graphs.erase(fz_graphs.begin());
        }
        hipGraph_t graph = nullptr;
        HIPCK(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed));
        try {
          enqueue();
        } catch (...) {
          (void)hipStreamEndCapture(stream, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          throw;
        }
        HIPCK(hipStreamEndCapture(stream, &graph));
        hipGraphExec_t exec = nullptr;
        const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCK(ie);
        fz_graphs.push_back(FzGraph{std::move(key), exec});
        g = &fz_graphs.back();
        ++fz_captures;
      }
      HIPCK(hipGraphLaunch(g->exec, stream));
    } else {
      enqueue();
    }
    mark(-1);
    sync();
    collect();
    if (h_fz[hl::kFusedOverflow] != 0) {
      u64 sum = 0;
      for (int r : idbs) sum += rels[r].n_delta;
      fz_fail_at = std::min(fz_fail_at, sum);
      fz_live = false;
      ++fz_overflows;
      return false;
    }
    ++fz_iterations;
    u64 in = 0, out = 0, d = 0;
    for (size_t r = 0; r < idbs.size(); ++r) {
      Relation& R = rels[idbs[r]];
      const u64* c = h_fz + r * hl::kFusedSlots;
      in += R.n_delta;
      out += c[5];
      st.candidates += c[4];
      st.join_outputs += c[5];
      R.delta_counts.push_back(c[2]);
      R.new_counts.push_back(c[3]);
      R.raw_cand = 0;
      R.n_cand = 0;
      std::swap(R.delta, R.fz_next);
      R.n_delta = c[2];
      if (c[2] > 0) {
        std::swap(R.fz_tail[0], R.fz_tail[1]);
        R.n_tail += c[2];
      }
      d += c[2];
    }
    last_in = in;
    last_out = out;
    fz_live = true;
    *total = d;
    return true;
  }

  template <typename K>
  void run_typed() {
    mark(HL_PHASE_INDEX_EDB);
    load_edbs<K>();
    mark(HL_PHASE_JOIN);
    for (const Plan& p : plans0) run_plan<K>(p);
    for (const WPlan& p : wplans0) run_wide_plan<K>(p);
    u64 d = close_iteration<K>();
    st.iterations = 1;
    if (fused_on()) fused_setup<K>();
    while (d != 0) {
      if (fused_next(d)) {
        u64 t = 0;
        if (fused_iteration<K>(&t)) {
          d = t;
          ++st.iterations;
          continue;
        }
      }
      fz_live = false;
      u64 in = 0;
      for (const Plan& p : plansR) in += rels[p.outer_rel].n_delta;
      for (const WPlan& p : wplansR) in += rels[p.outer_rel].n_delta;
      const u64 out0 = st.join_outputs;
      mark(HL_PHASE_JOIN);
      for (const Plan& p : plansR) run_plan<K>(p);
      for (const WPlan& p : wplansR) run_wide_plan<K>(p);
      last_in = in;
      last_out = st.join_outputs - out0;
      d = close_iteration<K>();
      ++st.iterations;
    }
    flush_tails<K>();
    sync();
    collect();
  }

  // ------------------------------------------------------------ autotune
  struct Setting {
    float lf, k;
    u32 fl;  // kTunedFlags bits
    int items;  // join expand outputs per thread
    int sort_items = 32;  // radix sort keys per thread of a tile
    int diff_items = 16;  // set difference candidates per thread of a tile
  };
  static constexpr u32 kTunedFlags = HL_FLAG_LEARNED_INDEX | HL_FLAG_JOIN_DEDUP | HL_FLAG_FUSED |
                                     HL_FLAG_HIP_GRAPH | HL_FLAG_NESTED_JOINS;

  void apply(const Setting& t) {
    load_factor = t.lf;
    ebm_k = t.k;
    flags = (flags & ~kTunedFlags) | t.fl;
    join_items = t.items;
    sort_items = t.sort_items;
    diff_items = t.diff_items;
  }

  // Fastest of `reps` timed runs after a warm-up; +inf if the device ran
  // out of memory.  The per-iteration delta sizes go to *deltas.
  double trial(const Setting& t, u32 reps, std::vector<std::vector<u64>>* deltas) {
    apply(t);
    hl_stats st{};
    double best = std::numeric_limits<double>::infinity();
    try {
      run(&st);
      for (u32 r = 0; r < reps; ++r) {
        run(&st);
        best = std::min(best, st.seconds);
      }
    } catch (const Error& x) {
      if (x.code != HL_E_NOMEM) throw;
      return std::numeric_limits<double>::infinity();
    }
    deltas->clear();
    for (const Relation& R : rels)
      if (!R.edb) deltas->push_back(R.delta_counts);
    return best;
  }

  void autotune(u32 reps, hl_tuning* out) {
    if (rules.empty()) fail(HL_E_STATE, "no program");
    Setting best{load_factor, ebm_k, flags & kTunedFlags, join_items, sort_items, diff_items};
    std::vector<std::vector<u64>> ref, got;
    u32 trials = 1;
    double best_t = trial(best, reps, &ref);
    const double first_t = best_t;
    bool have_ref = best_t < std::numeric_limits<double>::infinity();
    auto consider = [&](const Setting& t) {
      ++trials;
      const double v = trial(t, reps, &got);
      if (v == std::numeric_limits<double>::infinity()) return;
      if (!have_ref) {
        ref = got;
        have_ref = true;
      } else if (got != ref) {
        fail(HL_E_STATE, "autotune: settings gave different per-iteration deltas");
      }
      if (v < best_t) {
        best_t = v;
        best = t;
      }
    };
    // 1. how join inners are probed
    const Setting base = best;
    for (const Setting& t :
         {Setting{0.5f, base.k, base.fl & ~u32(HL_FLAG_LEARNED_INDEX), base.items,
                  base.sort_items, base.diff_items},
          Setting{0.8f, base.k, base.fl & ~u32(HL_FLAG_LEARNED_INDEX), base.items,
                  base.sort_items, base.diff_items},
          Setting{base.lf, base.k, base.fl | HL_FLAG_LEARNED_INDEX, base.items, base.sort_items,
                  base.diff_items}})
      if (t.lf != base.lf || t.fl != base.fl) consider(t);
    // join expand tile: outputs per thread
    {
      const Setting b = best;
      for (int it : {4, 8, 16}) {
        Setting t = b;
        t.items = it;
        if (it != b.items) consider(t);
      }
    }
    // radix sort tile (4,096 or 8,192 keys) and set difference tile (2,048
    // or 4,096 candidates)
    {
      Setting t = best;
      t.sort_items = best.sort_items == 32 ? 16 : 32;
      consider(t);
    }
    {
      Setting t = best;
      t.diff_items = best.diff_items == 16 ? 8 : 16;
      consider(t);
    }
    // 2. eager buffer growth factor
    {
      Setting t = best;
      t.k = best.k > 4.0f ? 1.5f : 8.0f;
      consider(t);
    }
    // 3. in-tile dedup of join outputs
    {
      Setting t = best;
      t.fl ^= HL_FLAG_JOIN_DEDUP;
      consider(t);
    }
    // 4. nested evaluation of two-join bodies (only where there are some)
    {
      bool two = false;
      for (auto* ps : {&plans0, &plansR})
        for (const Plan& p : *ps) two |= p.steps.size() == 2;
      if (two) {
        Setting t = best;
        t.fl ^= HL_FLAG_NESTED_JOINS;
        consider(t);
      }
    }
    // 5. fused small iterations, launched directly or from a HIP graph
    // (only where the recursive plans qualify)
    if (fz_plans && !(flags & HL_FLAG_NO_EBM)) {
      const Setting b = best;
      const u32 fz = HL_FLAG_FUSED | HL_FLAG_HIP_GRAPH;
      for (u32 f : {0u, u32(HL_FLAG_FUSED), fz}) {
        Setting t = b;
        t.fl = (b.fl & ~fz) | f;
        if (t.fl != b.fl) consider(t);
      }
    }
    if (!have_ref) fail(HL_E_NOMEM, "autotune: every setting ran out of device memory");
    apply(best);
    hl_stats st{};
    run(&st);
    if (out) {
      out->hash_load_factor = best.lf;
      out->ebm_k = best.k;
      out->flags = best.fl;
      out->trials = trials;
      out->expand_tile = u32(256 * best.items);
      out->sort_tile = u32(256 * best.sort_items);
      out->diff_tile = u32(256 * best.diff_items);
      out->best_seconds = best_t;
      out->first_seconds = first_t;
    }
  }

  void run(hl_stats* out) {
    if (rules.empty()) fail(HL_E_STATE, "no program");
    auto t0 = std::chrono::steady_clock::now();
    st = hl_stats{};
    rule_out.assign(rules.size(), 0);
    rule_mid.assign(rules.size(), 0);
    reuses = 0;
    fz_live = false;
    fz_fail_at = ~u64(0);
    last_in = last_out = 0;
    fz_iterations = fz_captures = fz_overflows = 0;
    drop_graphs();
    ktimer.reset();
    mem.reset_counters();
    marks.clear();
    ev_used = 0;
    for (Relation& R : rels) {
      R.delta_counts.clear();
      R.new_counts.clear();
      R.n_delta = R.n_cand = 0;
      R.n_tail = 0;
      R.lockstep_share = 0;
      R.dedup = true;
      R.raw_cand = 0;
      R.idx[0].lm_ok = R.idx[1].lm_ok = false;
      for (Index& ix : R.widx) ix.lm_ok = false;
      for (Index& tx : R.tidx) {
        tx.n = tx.cap = 0;
        tx.lm_ok = false;
      }
      if (!R.edb) {
        R.n_full = 0;
        R.idx[0].n = R.idx[1].n = 0;
        R.idx[0].cap = R.idx[1].cap = 0;
        for (Index& ix : R.widx) ix.n = ix.cap = 0;
      }
    }
    // key width: ids of every IDB tuple come from the EDBs (range restriction)
    HIPCK(hl::fill_zero(d_small, sizeof(u64), stream));
    for (Relation& R : rels)
      if (R.edb && R.n_raw)
        HIPCK(hl::max_u32(static_cast<const u32*>(R.raw.p), R.n_raw * R.arity,
                          reinterpret_cast<u32*>(d_small), stream));
    HIPCK(hipMemcpyAsync(h_small, d_small, sizeof(u64), hipMemcpyDeviceToHost, stream));
    sync();
    const u32 maxid = u32(h_small[0]);
    w = 1;
    while (w < 32 && (u64(maxid) >> w) != 0) ++w;
    const int cols = wide ? wide_cols() : 2;
    if (cols * w > 64)
      fail(HL_E_UNSUPPORTED, "tuples of " + std::to_string(cols) + " columns of " +
                                 std::to_string(w) + "-bit ids need keys wider than 64 bits");
    key_bytes = (cols * w <= 32) ? 4 : 8;
    if (key_bytes == 4) run_typed<u32>();
    else run_typed<u64>();
    st.key_bytes = key_bytes;
    st.id_bits = w;
    st.fused_iterations = u32(fz_iterations);
    st.fused_overflows = u32(fz_overflows);
    st.graph_captures = u32(fz_captures);
    for (Relation& R : rels)
      if (!R.edb) st.idb_tuples += R.n_full;
    st.peak_bytes = mem.peak();
    st.allocations = mem.allocs();
    st.ebm_reuses = reuses;
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    ran = true;
    if (out) *out = st;
  }

  template <typename K>
  void fetch_typed(Relation& R, u64 first, u64 count, u32* d_rows, u32 sub) {
    if (wide)
      HIPCK(hl::wide_unpack<K>(kp<K>(R.full) + first, count, R.arity, w, d_rows, stream, sub));
    else
      HIPCK(hl::unpack_rows<K>(kp<K>(R.full) + first, count, R.arity, w, d_rows, stream, sub));
  }

  // Tuples of relation R whose first column lies in [lo, hi): a contiguous
  // range of the sorted full relation (device search, one sync).
  template <typename K>
  std::pair<u64, u64> range_typed(Relation& R, u64 lo, u64 hi) {
    if (R.n_full == 0) return {0, 0};
    const u64 top = u64(1) << w;
    if (lo >= top) return {R.n_full, R.n_full};  // no id of the range occurs
    const K klo = lo >= top ? ~K(0) : K(K(lo) << w);
    const K khi = hi >= top ? ~K(0) : K(K(hi) << w);
    HIPCK(hl::key_range<K>(kp<K>(R.full), R.n_full, klo, khi, d_small, stream));
    HIPCK(hipMemcpyAsync(h_small, d_small, 2 * sizeof(u64), hipMemcpyDeviceToHost, stream));
    sync();
    u64 a = h_small[0], b = h_small[1];
    if (hi >= top) b = R.n_full;
    return {a, b};
  }

  std::pair<u64, u64> instance_range(Relation& R, u32 inst) {
    if (batch_base.empty()) fail(HL_E_STATE, "no batch layout");
    if (inst + 1 >= batch_base.size()) fail(HL_E_INVALID, "instance out of range");
    if (!ran) fail(HL_E_STATE, "fetch before hl_run");
    const u64 lo = batch_base[inst], hi = batch_base[inst + 1];
    return key_bytes == 4 ? range_typed<u32>(R, lo, hi) : range_typed<u64>(R, lo, hi);
  }

  void fetch_instance(const char* name, u32 inst, u32* rows, u64 cap, u64* n_rows) {
    Relation& R = rels[find_or_fail(name)];
    auto rg = instance_range(R, inst);
    const u64 cnt = rg.second - rg.first;
    if (n_rows) *n_rows = cnt;
    if (cap < cnt) fail(HL_E_CAPACITY, "buffer holds " + std::to_string(cap) + " rows, need " +
                                          std::to_string(cnt));
    if (cnt == 0) return;
    if (!rows) fail(HL_E_INVALID, "null output buffer");
    const u64 bytes = cnt * R.arity * sizeof(u32);
    reserve_grow(this->rows, bytes);
    u32* dst = static_cast<u32*>(this->rows.p);
    const u32 sub = u32(batch_base[inst]);
    if (key_bytes == 4) fetch_typed<u32>(R, rg.first, cnt, dst, sub);
    else fetch_typed<u64>(R, rg.first, cnt, dst, sub);
    HIPCK(hipMemcpyAsync(rows, dst, bytes, hipMemcpyDeviceToHost, stream));
    sync();
  }

  void fetch(const char* name, u32* rows, u64 cap, u64* n_rows, bool device) {
    Relation& R = rels[find_or_fail(name)];
    if (!ran) fail(HL_E_STATE, "fetch before hl_run");
    if (n_rows) *n_rows = R.n_full;
    if (cap < R.n_full) fail(HL_E_CAPACITY, "buffer holds " + std::to_string(cap) + " rows, need " +
                                               std::to_string(R.n_full));
    if (R.n_full == 0) return;
    if (!rows) fail(HL_E_INVALID, "null output buffer");
    const u64 bytes = R.n_full * R.arity * sizeof(u32);
    u32* dst;
    if (device) {
      dst = rows;
    } else {
      reserve_grow(this->rows, bytes);
      dst = static_cast<u32*>(this->rows.p);
    }
    if (key_bytes == 4) fetch_typed<u32>(R, 0, R.n_full, dst, 0);
    else fetch_typed<u64>(R, 0, R.n_full, dst, 0);
    if (!device) HIPCK(hipMemcpyAsync(rows, dst, bytes, hipMemcpyDeviceToHost, stream));
    sync();
  }
};

// ---------------------------------------------------------------- C ABI

namespace {

template <typename F>
int guard(hl_engine* e, F&& f) {
  if (!e) return HL_E_INVALID;
  try {
    if (e->device >= 0) HIPCK(hipSetDevice(e->device));
    f();
    e->err.clear();
    return HL_OK;
  } catch (const Error& x) {
    e->err = x.msg;
    return x.code;
  } catch (const std::bad_alloc&) {
    e->err = "host out of memory";
    return HL_E_NOMEM;
  } catch (...) {
    e->err = "unexpected internal error";
    return HL_E_INVALID;
  }
}

bool valid_key_bytes(u32 kb) { return kb == 4 || kb == 8; }

}  // namespace

extern "C" {

int hl_options_init(hl_options* opt) {
  if (!opt) return HL_E_INVALID;
  memset(opt, 0, sizeof(*opt));
  opt->ebm_k = 8.0f;
  opt->hash_load_factor = 0.5f;
  return HL_OK;
}

int hl_create(const hl_options* opt, hl_engine** out) {
  if (!out) return HL_E_INVALID;
  *out = nullptr;
  hl_options o;
  hl_options_init(&o);
  if (opt) o = *opt;
  if (!(o.ebm_k >= 1.0f) || !(o.hash_load_factor > 0.0f && o.hash_load_factor <= 1.0f))
    return HL_E_INVALID;
  if (o.outer_slice_log2 != 0 && (o.outer_slice_log2 < 8 || o.outer_slice_log2 > 31))
    return HL_E_INVALID;
  if (o.arena && o.arena_bytes < 4096) return HL_E_INVALID;
  if (o.sort_chunk_log2 != 0 && (o.sort_chunk_log2 < 12 || o.sort_chunk_log2 > 31))
    return HL_E_INVALID;
  if (o.fused_capacity != 0 &&
      (o.fused_capacity < 1024 || (o.fused_capacity & (o.fused_capacity - 1)) != 0))
    return HL_E_INVALID;
  if (o.expand_tile != 0 && o.expand_tile != 1024 && o.expand_tile != 2048 &&
      o.expand_tile != 4096)
    return HL_E_INVALID;
  if (o.sort_tile != 0 && o.sort_tile != 4096 && o.sort_tile != 8192) return HL_E_INVALID;
  if (o.diff_tile != 0 && o.diff_tile != 2048 && o.diff_tile != 4096) return HL_E_INVALID;
  if (o.device == -1) {
    // planning-only engine: declarations and programs, no device work
    hl_engine* e = new (std::nothrow) hl_engine();
    if (!e) return HL_E_NOMEM;
    e->device = -1;
    *out = e;
    return HL_OK;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || o.device < 0 || o.device >= ndev) {
    (void)hipGetLastError();
    return HL_E_DEVICE;
  }
  hl_engine* e = new (std::nothrow) hl_engine();
  if (!e) return HL_E_NOMEM;
  e->device = o.device;
  e->flags = o.flags;
  e->ebm_k = o.ebm_k;
  e->load_factor = o.hash_load_factor;
  e->sort_chunk_log2 = int(o.sort_chunk_log2);
  e->fused_capacity = o.fused_capacity;
  e->join_items = o.expand_tile ? int(o.expand_tile / 256) : 8;
  e->sort_items = o.sort_tile ? int(o.sort_tile / 256) : 32;
  e->tail_min_bytes = o.tail_min_bytes ? o.tail_min_bytes : hl_engine::kTailMinFullBytes;
  e->outer_slice = u64(1) << (o.outer_slice_log2 ? o.outer_slice_log2 : 28);
  e->diff_items = o.diff_tile ? int(o.diff_tile / 256) : 16;
  int rc = guard(e, [&] {
    if (o.stream) {
      e->stream = static_cast<hipStream_t>(o.stream);
    } else {
      HIPCK(hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking));
      e->own_stream = true;
    }
    // the device address of the static scratch (the device is current
    // here); hl_sort_keys_noalloc passes only this address to kernels
    HIPCK(hl::noalloc_scratch(e->device, &e->noalloc));
    e->mem.init(o.arena, o.arena_bytes, o.hbm_budget_bytes, e->stream);
    e->mem.set_caching(!(o.flags & HL_FLAG_NO_EBM));
    e->d_small = static_cast<u64*>(e->mem.alloc(hl_engine::kSmall * sizeof(u64)));
    HIPCK(hipHostMalloc(reinterpret_cast<void**>(&e->h_small), hl_engine::kSmall * sizeof(u64),
                        hipHostMallocDefault));
    e->d_fz = static_cast<u64*>(e->mem.alloc(hl::kFusedCountWords * sizeof(u64)));
    HIPCK(hipHostMalloc(reinterpret_cast<void**>(&e->h_fz), hl::kFusedCountWords * sizeof(u64),
                        hipHostMallocDefault));
  });
  if (rc != HL_OK) {
    hl_destroy(e);
    return rc;
  }
  *out = e;
  return HL_OK;
}

void hl_destroy(hl_engine* e) {
  if (!e) return;
  if (e->device < 0) {
    delete e;
    return;
  }
  (void)hipSetDevice(e->device);
  if (e->stream) (void)hipStreamSynchronize(e->stream);
  e->drop_graphs();
  e->mem.release_all();
  for (hipEvent_t ev : e->ev_pool) (void)hipEventDestroy(ev);
  if (e->h_small) (void)hipHostFree(e->h_small);
  if (e->h_fz) (void)hipHostFree(e->h_fz);
  if (e->own_stream && e->stream) (void)hipStreamDestroy(e->stream);
  delete e;
}

int hl_declare(hl_engine* e, const char* name, uint32_t arity, int32_t is_edb) {
  return guard(e, [&] {
    if (!name || !*name || strlen(name) > 63) fail(HL_E_INVALID, "bad relation name");
    for (const char* c = name; *c; ++c)
      if (!(isalnum(static_cast<unsigned char>(*c)) || *c == '_'))
        fail(HL_E_INVALID, "bad relation name");
    if (!e->rules.empty()) fail(HL_E_STATE, "declare before hl_program");
    if (e->find(name) >= 0) fail(HL_E_INVALID, std::string("relation declared twice: ") + name);
    if (arity < 1 || arity > 4) fail(HL_E_UNSUPPORTED, "relations of arity 1 to 4 only");
    Relation R;
    R.name = name;
    R.arity = int(arity);
    R.edb = is_edb != 0;
    e->rels.push_back(R);
  });
}

static int load_impl(hl_engine* e, const char* name, const uint32_t* rows, uint64_t n, bool dev) {
  return guard(e, [&] {
    if (e->device < 0) fail(HL_E_STATE, "planning-only engine (device -1)");
    Relation& R = e->rels[e->find_or_fail(name)];
    if (!R.edb) fail(HL_E_INVALID, "load into an IDB relation");
    if (n == 0) return;
    if (!rows) fail(HL_E_INVALID, "null rows");
    const u64 row_bytes = u64(R.arity) * sizeof(u32);
    const u64 total = R.n_raw + n;
    if (total >= (u64(1) << 32)) fail(HL_E_UNSUPPORTED, "EDB relation with 2^32 or more rows");
    Buf nb;
    nb.p = e->mem.alloc(total * row_bytes);
    nb.bytes = total * row_bytes;
    if (R.n_raw)
      HIPCK(hipMemcpyAsync(nb.p, R.raw.p, R.n_raw * row_bytes, hipMemcpyDeviceToDevice, e->stream));
    HIPCK(hipMemcpyAsync(static_cast<char*>(nb.p) + R.n_raw * row_bytes, rows, n * row_bytes,
                         dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, e->stream));
    if (!dev) e->sync();  // the caller may reuse its host buffer on return
    e->drop(R.raw);
    R.raw = nb;
    R.n_raw = total;
  });
}

int hl_load(hl_engine* e, const char* name, const uint32_t* rows, uint64_t n_rows) {
  return load_impl(e, name, rows, n_rows, false);
}

int hl_load_device(hl_engine* e, const char* name, const uint32_t* d_rows, uint64_t n_rows) {
  return load_impl(e, name, d_rows, n_rows, true);
}

int hl_batch_layout(hl_engine* e, const uint32_t* id_range, uint32_t n_inst) {
  return guard(e, [&] {
    if (!id_range || n_inst == 0) fail(HL_E_INVALID, "empty batch layout");
    if (!e->batch_base.empty()) fail(HL_E_STATE, "batch layout already set");
    for (const Relation& R : e->rels) {
      if (R.n_raw) fail(HL_E_STATE, "batch layout after rows were loaded");
      if (R.arity > 2) fail(HL_E_UNSUPPORTED, "batches of relations of arity above 2");
    }
    if (e->wide) fail(HL_E_UNSUPPORTED, "batches of wide programs");
    std::vector<u64> base(n_inst + 1, 0);
    for (u32 k = 0; k < n_inst; ++k) base[k + 1] = base[k] + id_range[k];
    if (base[n_inst] > (u64(1) << 32)) fail(HL_E_INVALID, "instance id ranges exceed 2^32");
    e->batch_base = base;
  });
}

int hl_load_batched(hl_engine* e, const char* name, const uint32_t* rows,
                    const uint64_t* inst_offsets) {
  int rc = guard(e, [&] {
    if (e->batch_base.empty()) fail(HL_E_STATE, "hl_batch_layout first");
    Relation& R = e->rels[e->find_or_fail(name)];
    if (!R.edb) fail(HL_E_INVALID, "load into an IDB relation");
    if (!inst_offsets) fail(HL_E_INVALID, "null offsets");
    const u32 ni = u32(e->batch_base.size() - 1);
    if (inst_offsets[0] != 0) fail(HL_E_INVALID, "offsets must start at 0");
    for (u32 k = 0; k < ni; ++k)
      if (inst_offsets[k + 1] < inst_offsets[k]) fail(HL_E_INVALID, "offsets must not decrease");
    const u64 n = inst_offsets[ni];
    if (n && !rows) fail(HL_E_INVALID, "null rows");
    // dictionary encoding: instance k's id v becomes base[k] + v
    std::vector<u32> mapped(n * R.arity);
    for (u32 k = 0; k < ni; ++k) {
      const u64 b = e->batch_base[k], range = e->batch_base[k + 1] - b;
      for (u64 i = inst_offsets[k] * R.arity; i < inst_offsets[k + 1] * R.arity; ++i) {
        if (rows[i] >= range) fail(HL_E_INVALID, "id outside its instance's range");
        mapped[i] = u32(b + rows[i]);
      }
    }
    e->batch_rows_tmp.swap(mapped);
  });
  if (rc != HL_OK) return rc;
  std::vector<u32> mapped;
  mapped.swap(e->batch_rows_tmp);
  // rows of the relation's declared arity (the guard above found it)
  const u64 n = mapped.size() / u64(e->rels[e->find(name)].arity);
  return hl_load(e, name, mapped.data(), n);
}

int hl_batch_count(hl_engine* e, const char* name, uint32_t inst, uint64_t* n) {
  return guard(e, [&] {
    if (!n) fail(HL_E_INVALID, "null output");
    Relation& R = e->rels[e->find_or_fail(name)];
    auto rg = e->instance_range(R, inst);
    *n = rg.second - rg.first;
  });
}

int hl_fetch_batched(hl_engine* e, const char* name, uint32_t inst, uint32_t* rows,
                     uint64_t cap_rows, uint64_t* n_rows) {
  return guard(e, [&] { e->fetch_instance(name, inst, rows, cap_rows, n_rows); });
}

int hl_index(hl_engine* e, const char* name, const uint32_t* cols, uint32_t ncols) {
  return guard(e, [&] {
    Relation& R = e->rels[e->find_or_fail(name)];
    if (!cols || ncols != 1) fail(HL_E_UNSUPPORTED, "indexes on one column only");
    if (cols[0] >= u32(R.arity)) fail(HL_E_INVALID, "column out of range");
    if (R.arity > 2)
      fail(HL_E_UNSUPPORTED, "relations of arity 3-4 get the indexes their joins need");
    R.idx[cols[0]].used = true;
  });
}

int hl_program(hl_engine* e, const char* text) {
  return guard(e, [&] {
    if (!text) fail(HL_E_INVALID, "null program");
    std::vector<Rule> parsed = e->parse(text);
    std::vector<Rule> saved = e->rules;
    e->rules.insert(e->rules.end(), parsed.begin(), parsed.end());
    try {
      e->build_plans();
    } catch (...) {
      e->rules = saved;
      throw;
    }
  });
}

int hl_run(hl_engine* e, hl_stats* stats) {
  return guard(e, [&] {
    if (e->device < 0) fail(HL_E_STATE, "planning-only engine (device -1)");
    e->run(stats);
  });
}

int hl_rule_stats(hl_engine* e, uint32_t rule, uint64_t* join_outputs, uint64_t* intermediate) {
  return guard(e, [&] {
    if (!join_outputs || !intermediate) fail(HL_E_INVALID, "null output");
    if (!e->ran) fail(HL_E_STATE, "rule statistics before hl_run");
    if (rule >= e->rule_out.size()) fail(HL_E_INVALID, "no such rule");
    *join_outputs = e->rule_out[rule];
    *intermediate = e->rule_mid[rule];
  });
}

int hl_autotune(hl_engine* e, uint32_t reps, hl_tuning* out) {
  return guard(e, [&] {
    if (e->device < 0) fail(HL_E_STATE, "planning-only engine (device -1)");
    e->autotune(reps < 1 ? 1 : reps, out);
  });
}

int hl_count(hl_engine* e, const char* name, uint64_t* n) {
  return guard(e, [&] {
    if (!n) fail(HL_E_INVALID, "null output");
    Relation& R = e->rels[e->find_or_fail(name)];
    if (!e->ran) fail(HL_E_STATE, "count before hl_run");
    *n = R.n_full;
  });
}

int hl_fetch(hl_engine* e, const char* name, uint32_t* rows, uint64_t cap_rows,
             uint64_t* n_rows) {
  return guard(e, [&] { e->fetch(name, rows, cap_rows, n_rows, false); });
}

int hl_fetch_device(hl_engine* e, const char* name, uint32_t* d_rows, uint64_t cap_rows,
                    uint64_t* n_rows) {
  return guard(e, [&] { e->fetch(name, d_rows, cap_rows, n_rows, true); });
}

int hl_iteration_counts(hl_engine* e, const char* name, int32_t which, uint64_t* counts,
                        uint32_t cap, uint32_t* n_iters) {
  return guard(e, [&] {
    Relation& R = e->rels[e->find_or_fail(name)];
    if (which != 0 && which != 1) fail(HL_E_INVALID, "which must be 0 or 1");
    const std::vector<u64>& v = which == 0 ? R.delta_counts : R.new_counts;
    if (n_iters) *n_iters = u32(v.size());
    for (u32 i = 0; i < cap && i < v.size(); ++i) counts[i] = v[i];
  });
}

int hl_kernel_stats(hl_engine* e, int32_t kernel, uint64_t* launches, double* ms,
                    uint64_t* algorithmic_bytes) {
  return guard(e, [&] {
    if (kernel < 0 || kernel >= hl::K_COUNT) fail(HL_E_INVALID, "unknown kernel id");
    const EventTimer::Total& t = e->ktimer.totals[kernel];
    if (launches) *launches = t.launches;
    if (ms) *ms = t.ms;
    if (algorithmic_bytes) *algorithmic_bytes = t.bytes;
  });
}

const char* hl_last_error(hl_engine* e) { return e ? e->err.c_str() : "null engine"; }

const char* hl_strerror(int code) {
  switch (code) {
    case HL_OK: return "ok";
    case HL_E_INVALID: return "invalid argument";
    case HL_E_NOMEM: return "out of device memory";
    case HL_E_DEVICE: return "HIP runtime error";
    case HL_E_STATE: return "call not allowed in this state";
    case HL_E_CAPACITY: return "output buffer too small";
    case HL_E_UNSUPPORTED: return "unsupported";
    default: return "unknown error";
  }
}

// ------------------------------------------------------------ primitives

int hl_sort_keys(hl_engine* e, void* d_keys, uint64_t n, uint32_t key_bytes, uint32_t bits) {
  return guard(e, [&] {
    if (e->device < 0) fail(HL_E_STATE, "planning-only engine (device -1)");
    if (!valid_key_bytes(key_bytes)) fail(HL_E_INVALID, "key_bytes must be 4 or 8");
    if (n >= (u64(1) << 32)) fail(HL_E_UNSUPPORTED, "2^32 or more keys");
    if (n <= 1) return;
    if (!d_keys) fail(HL_E_INVALID, "null keys");
    int b = bits ? int(bits) : int(8 * key_bytes);
    if (b > int(8 * key_bytes)) fail(HL_E_INVALID, "bits exceed the key width");
    e->reserve_grow(e->alt, n * key_bytes);
    e->reserve(e->ws, hl::sort_workspace_bytes(n), hl::sort_workspace_bytes(n));
    void* sorted = nullptr;
    if (key_bytes == 4) {
      u32* s = nullptr;
      HIPCK(hl::radix_sort<u32>(static_cast<u32*>(d_keys), static_cast<u32*>(e->alt.p), n, b,
                                e->ws.p, e->stream, &s, nullptr));
      sorted = s;
    } else {
      u64* s = nullptr;
      HIPCK(hl::radix_sort<u64>(static_cast<u64*>(d_keys), static_cast<u64*>(e->alt.p), n, b,
                                e->ws.p, e->stream, &s, nullptr));
      sorted = s;
    }
    if (sorted != d_keys)
      HIPCK(hipMemcpyAsync(d_keys, sorted, n * key_bytes, hipMemcpyDeviceToDevice, e->stream));
    e->sync();
  });
}

int hl_sort_keys_noalloc(hl_engine* e, void* d_keys, uint64_t n, uint32_t key_bytes,
                         uint32_t bits) {
  return guard(e, [&] {
    if (e->device < 0) fail(HL_E_STATE, "planning-only engine (device -1)");
    if (!valid_key_bytes(key_bytes)) fail(HL_E_INVALID, "key_bytes must be 4 or 8");
    const int b = bits ? int(bits) : int(8 * key_bytes);
    if (b > int(8 * key_bytes)) fail(HL_E_INVALID, "bits exceed the key width");
    if (n <= 1) return;
    if (!d_keys) fail(HL_E_INVALID, "null keys");
    // the second buffer of the sort, then its count matrices
    const u64 room = hl::noalloc_scratch_bytes();
    const u64 alt_bytes = hl::align_up(n * key_bytes, 256);
    if (n >= room || alt_bytes + hl::sort_workspace_bytes(n) > room)
      fail(HL_E_CAPACITY, std::to_string(n) + " keys of " + std::to_string(key_bytes) +
                              " bytes need more than the " + std::to_string(room >> 20) +
                              " MiB of static scratch");
    if (!e->noalloc) fail(HL_E_STATE, "no static scratch on this device");
    char* sc = static_cast<char*>(e->noalloc);
    void* sorted = nullptr;
    if (key_bytes == 4) {
      u32* s = nullptr;
      HIPCK(hl::radix_sort<u32>(static_cast<u32*>(d_keys), reinterpret_cast<u32*>(sc), n, b,
                                sc + alt_bytes, e->stream, &s, nullptr));
      sorted = s;
    } else {
      u64* s = nullptr;
      HIPCK(hl::radix_sort<u64>(static_cast<u64*>(d_keys), reinterpret_cast<u64*>(sc), n, b,
                                sc + alt_bytes, e->stream, &s, nullptr));
      sorted = s;
    }
    if (sorted != d_keys)
      HIPCK(hipMemcpyAsync(d_keys, sorted, n * key_bytes, hipMemcpyDeviceToDevice, e->stream));
    e->sync();
  });
}

int hl_unique_diff(hl_engine* e, const void* d_sorted, uint64_t n, const void* d_full,
                   uint64_t n_full, void* d_out, uint64_t* n_out, uint64_t* n_unique,
                   uint32_t key_bytes) {
  return guard(e, [&] {
    if (e->device < 0) fail(HL_E_STATE, "planning-only engine (device -1)");
    if (!valid_key_bytes(key_bytes)) fail(HL_E_INVALID, "key_bytes must be 4 or 8");
    if (n >= (u64(1) << 32)) fail(HL_E_UNSUPPORTED, "2^32 or more keys");
    if ((n && (!d_sorted || !d_out)) || (n_full && !d_full)) fail(HL_E_INVALID, "null buffer");
    e->reserve_grow(e->alt, std::max<u64>(n, 1) * key_bytes);
    e->reserve(e->ws, hl::unique_diff_workspace_bytes(n), hl::unique_diff_workspace_bytes(n));
    if (key_bytes == 4)
      HIPCK(hl::unique_diff<u32>(static_cast<const u32*>(d_sorted), n,
                                 static_cast<const u32*>(d_full), n_full,
                                 static_cast<u32*>(e->alt.p), static_cast<u32*>(d_out),
                                 e->d_small, e->ws.p, e->stream));
    else
      HIPCK(hl::unique_diff<u64>(static_cast<const u64*>(d_sorted), n,
                                 static_cast<const u64*>(d_full), n_full,
                                 static_cast<u64*>(e->alt.p), static_cast<u64*>(d_out),
                                 e->d_small, e->ws.p, e->stream));
    HIPCK(hipMemcpyAsync(e->h_small, e->d_small, 2 * sizeof(u64), hipMemcpyDeviceToHost,
                         e->stream));
    e->sync();
    if (n_out) *n_out = e->h_small[0];
    if (n_unique) *n_unique = e->h_small[1];
  });
}

int hl_merge(hl_engine* e, const void* d_a, uint64_t na, const void* d_b, uint64_t nb,
             void* d_out, uint32_t key_bytes) {
  return guard(e, [&] {
    if (e->device < 0) fail(HL_E_STATE, "planning-only engine (device -1)");
    if (!valid_key_bytes(key_bytes)) fail(HL_E_INVALID, "key_bytes must be 4 or 8");
    if ((na && !d_a) || (nb && !d_b) || (na + nb && !d_out)) fail(HL_E_INVALID, "null buffer");
    e->reserve(e->ws, hl::merge_workspace_bytes(na, nb), hl::merge_workspace_bytes(na, nb));
    if (key_bytes == 4)
      HIPCK(hl::merge<u32>(static_cast<const u32*>(d_a), na, static_cast<const u32*>(d_b), nb,
                           static_cast<u32*>(d_out), e->ws.p, e->stream));
    else
      HIPCK(hl::merge<u64>(static_cast<const u64*>(d_a), na, static_cast<const u64*>(d_b), nb,
                           static_cast<u64*>(d_out), e->ws.p, e->stream));
    e->sync();
  });
}

int hl_hisa_query(hl_engine* e, const void* d_keys, uint64_t n, uint32_t key_bytes,
                  uint32_t shift, const uint32_t* d_queries, uint64_t nq, uint64_t* d_start,
                  uint32_t* d_len, uint64_t* n_runs) {
  return guard(e, [&] {
    if (e->device < 0) fail(HL_E_STATE, "planning-only engine (device -1)");
    if (!valid_key_bytes(key_bytes)) fail(HL_E_INVALID, "key_bytes must be 4 or 8");
    if (n >= (u64(1) << 32)) fail(HL_E_UNSUPPORTED, "2^32 or more keys");
    if (shift >= 8 * key_bytes) fail(HL_E_INVALID, "shift out of range");
    if ((n && !d_keys) || (nq && (!d_queries || !d_start || !d_len)))
      fail(HL_E_INVALID, "null buffer");
    if (key_bytes == 4)
      HIPCK(hl::hisa_count_runs<u32>(static_cast<const u32*>(d_keys), n, int(shift), e->d_small,
                                     e->stream));
    else
      HIPCK(hl::hisa_count_runs<u64>(static_cast<const u64*>(d_keys), n, int(shift), e->d_small,
                                     e->stream));
    HIPCK(hipMemcpyAsync(e->h_small, e->d_small, sizeof(u64), hipMemcpyDeviceToHost, e->stream));
    e->sync();
    const u64 runs = e->h_small[0];
    if (n_runs) *n_runs = runs;
    u64 cap = std::max<u64>(u64(std::ceil(double(runs) / e->load_factor)), runs + 1);
    cap = std::max<u64>(cap, 16);
    Buf table;
    table.p = e->mem.alloc(cap * sizeof(Slot));
    table.bytes = cap * sizeof(Slot);
    try {
      HIPCK(hl::fill_zero(table.p, cap * sizeof(Slot), e->stream));
      if (key_bytes == 4)
        HIPCK(hl::hisa_build<u32>(static_cast<const u32*>(d_keys), n, int(shift),
                                  static_cast<Slot*>(table.p), cap, e->stream));
      else
        HIPCK(hl::hisa_build<u64>(static_cast<const u64*>(d_keys), n, int(shift),
                                  static_cast<Slot*>(table.p), cap, e->stream));
      HIPCK(hl::hisa_probe(static_cast<Slot*>(table.p), cap, d_queries, nq, d_start, d_len,
                           e->stream));
      e->sync();
    } catch (...) {
      e->drop(table);
      throw;
    }
    e->drop(table);
  });
}

int hl_learned_query(hl_engine* e, const void* d_keys, uint64_t n, uint32_t key_bytes,
                     uint32_t key_bits, const void* d_queries, uint64_t nq, uint32_t* d_pos) {
  return guard(e, [&] {
    if (e->device < 0) fail(HL_E_STATE, "planning-only engine (device -1)");
    if (!valid_key_bytes(key_bytes)) fail(HL_E_INVALID, "key_bytes must be 4 or 8");
    if (key_bits < 1 || key_bits > 8 * key_bytes) fail(HL_E_INVALID, "key_bits out of range");
    if (n >= (u64(1) << 32)) fail(HL_E_UNSUPPORTED, "2^32 or more keys");
    if ((n && !d_keys) || (nq && (!d_queries || !d_pos))) fail(HL_E_INVALID, "null buffer");
    const int bits = hl::learned_bits(n, int(key_bits));
    const u64 bytes = hl::learned_bytes(bits);
    Buf m;
    m.p = e->mem.alloc(bytes);
    m.bytes = bytes;
    try {
      if (key_bytes == 4) {
        hl::LearnedView<u32> v{};
        HIPCK(hl::learned_fit<u32>(static_cast<const u32*>(d_keys), n, int(key_bits), bits, m.p,
                                   e->stream, &v));
        HIPCK(hl::learned_query(v, static_cast<const u32*>(d_queries), nq, d_pos, e->stream));
      } else {
        hl::LearnedView<u64> v{};
        HIPCK(hl::learned_fit<u64>(static_cast<const u64*>(d_keys), n, int(key_bits), bits, m.p,
                                   e->stream, &v));
        HIPCK(hl::learned_query(v, static_cast<const u64*>(d_queries), nq, d_pos, e->stream));
      }
      e->sync();
    } catch (...) {
      e->drop(m);
      throw;
    }
    e->drop(m);
  });
}

}  // extern "C"
