// Host-side launchers of the gfx950 kernels.  Every launcher validates its
// sizes before it launches, enqueues on `s`, and returns the first HIP
// error.  Workspaces are caller-provided device memory of at least the
// size the matching *_workspace_bytes() function returns; nothing here
// allocates.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "learned.hpp"

namespace hl {

typedef uint32_t u32;
typedef uint64_t u64;

// One slot of the HISA hash index.  w0 = (run length << 32) | join key;
// w0 == 0 marks an empty slot (every stored run has length >= 1, so no
// stored slot is 0).  w1 = position of the run's first tuple in the
// sorted array.
struct alignas(16) Slot {
  u64 w0;
  u64 w1;
};

inline u64 align_up(u64 x, u64 a) { return (x + a - 1) / a * a; }

// Kernels whose launches can be timed one by one with HIP events.
enum KernelId {
  K_RADIX_HIST = 0,
  K_RADIX_SCATTER = 1,
  K_UNIQUE_DIFF = 2,
  K_MERGE = 3,
  K_JOIN_PROBE = 4,
  K_JOIN_EXPAND = 5,
  K_HISA_BUILD = 6,
  K_LEARNED_FIT = 7,
  K_COUNT = 8
};

// Optional launch timer: launchers call begin() right before and end()
// right after a timed kernel, passing the bytes the kernel must move by
// definition (its inputs read once, its outputs written once).
// A kernel whose byte count depends on what it finds (how many keys it
// keeps, how far apart its searches fall) adds that part on the device: the
// launcher asks for a counter (zeroed on the stream), the kernel adds to it,
// and end() takes it along with the part known on the host.
struct LaunchTimer {
  virtual void begin(int kernel, hipStream_t s) = 0;
  virtual void end(int kernel, hipStream_t s, u64 algorithmic_bytes,
                   const u64* device_bytes = nullptr) = 0;
  virtual u64* device_counter(hipStream_t) { return nullptr; }
  virtual ~LaunchTimer() {}
};

// ---------------------------------------------------------------- scan
u64 scan_workspace_bytes(u64 n);
// Exclusive prefix sum of u32 values into u64 offsets; *d_total (device)
// receives the sum.  In place (out aliasing in) is not allowed.
hipError_t scan_u32_u64(const u32* in, u64 n, u64* out, u64* d_total, void* ws, hipStream_t s);

// ---------------------------------------------------------- radix sort
// Workspace of a sort of n keys with any tile size.
u64 sort_workspace_bytes(u64 n);
// LSD radix sort of the low `bits` bits of n keys (the bits above must be
// zero).  Ping-pongs between `keys` and `alt`; *sorted receives whichever
// holds the result (the other one is free afterwards).  n must be below
// 2^32.  tile_items: keys per thread of a tile, 32 (8,192-key tiles) or 16.
template <typename K>
hipError_t radix_sort(K* keys, K* alt, u64 n, int bits, void* ws, hipStream_t s, K** sorted,
                      LaunchTimer* timer = nullptr, int tile_items = 32);
// Stable LSD radix sort on bits [lo_bit, hi_bit) of the keys only: keys
// equal on those bits keep their input order (used to group an array by one
// column).  Same buffers and limits as radix_sort.
template <typename K>
hipError_t radix_sort_bits(K* keys, K* alt, u64 n, int lo_bit, int hi_bit, void* ws,
                           hipStream_t s, K** sorted, LaunchTimer* timer = nullptr,
                           int tile_items = 32);

// --------------------------------------------- unique + set difference
u64 unique_diff_workspace_bytes(u64 n);
// out = unique(sorted) \ full.  Both inputs sorted ascending; full has no
// duplicates.  `tmp` holds n keys.  d_counts[0] = |out|, d_counts[1] =
// number of distinct keys in `sorted`.  n must be below 2^32.
// With `model` (a learned index over full), the slice of full each tile
// spans and the membership tests outside LDS go through the model.  With a
// tail (ntail sorted unique keys, disjoint from full), keys it holds are
// dropped too: the result is unique(sorted) \ (full U tail).
// `items`: candidates per thread of a tile, 16 (4,096-candidate tiles) or 8.
// With out == nullptr the survivors stay in tmp (compacted per tile) and
// unique_diff_gather, called with the same n, nf, ws and items before ws is
// reused, writes them to their final place once the caller knows the count.
// When full has no more keys than there are candidates (nf <= n) the tiles
// follow the merge path of the two arrays instead (items and the model do
// not apply).
// lockstep_tiles (device, optional): incremented once per tile whose slice
// of full is too long to stream (its keys are searched in global memory).
template <typename K>
hipError_t unique_diff(const K* sorted, u64 n, const K* full, u64 nf, K* tmp, K* out,
                       u64* d_counts, void* ws, hipStream_t s, LaunchTimer* timer = nullptr,
                       const LearnedView<K>* model = nullptr, const K* tail = nullptr,
                       u64 ntail = 0, int items = 16, u64* lockstep_tiles = nullptr);
template <typename K>
hipError_t unique_diff_gather(const K* tmp, u64 n, u64 nf, const void* ws, K* out,
                              hipStream_t s, int items = 16);

// --------------------------------------------------------------- merge
u64 merge_workspace_bytes(u64 na, u64 nb);
// out = merge of two ascending arrays (ties take a first).
template <typename K>
hipError_t merge(const K* a, u64 na, const K* b, u64 nb, K* out, void* ws, hipStream_t s,
                 LaunchTimer* timer = nullptr);

// ---------------------------------------------------------------- HISA
// Counts the runs of equal join key (key >> shift) of a sorted array.
template <typename K>
hipError_t hisa_count_runs(const K* keys, u64 n, int shift, u64* d_runs, hipStream_t s);
// Inserts every run into an open-addressing table of `cap` slots, which
// must exceed the number of runs and start zeroed (see fill_zero).
template <typename K>
hipError_t hisa_build(const K* keys, u64 n, int shift, Slot* table, u64 cap, hipStream_t s,
                      LaunchTimer* timer = nullptr);
// Looks up nq join keys; len 0 means absent.
hipError_t hisa_probe(const Slot* table, u64 cap, const u32* q, u64 nq, u64* start, u32* len,
                      hipStream_t s);

// -------------------------------------------------------- learned index
// Radix bits for an index over n keys of key_bits significant bits.
int learned_bits(u64 n, int key_bits);
u64 learned_bytes(int radix_bits);
// Fits the model of n sorted keys (n < 2^32) into `mem` (learned_bytes).
template <typename K>
hipError_t learned_fit(const K* keys, u64 n, int key_bits, int radix_bits, void* mem,
                       hipStream_t s, LearnedView<K>* out, LaunchTimer* timer = nullptr);
// out[i] = lower_bound(keys, q[i]) through the model.
hipError_t learned_query(const LearnedView<u32>& lv, const u32* q, u64 nq, u32* out,
                         hipStream_t s);
hipError_t learned_query(const LearnedView<u64>& lv, const u64* q, u64 nq, u32* out,
                         hipStream_t s);

// ------------------------------------------------- static scratch
// Bytes of the file-scope device array behind the entry point that
// allocates nothing (noalloc.hip).
u64 noalloc_scratch_bytes();
// With `device` current: that device's address of the array (looked up
// with hipGetSymbolAddress on the first call for the device, then kept).
hipError_t noalloc_scratch(int device, void** ptr);

// ---------------------------------------------------------------- misc
hipError_t fill_zero(void* p, u64 bytes, hipStream_t s);
// *d_max = max(*d_max, v[i]); *d_max must be initialised.
hipError_t max_u32(const u32* v, u64 n, u32* d_max, hipStream_t s);
// Row-major uint32 pairs -> keys (c0 << w) | c1; arity 1 packs (c0 << w).
template <typename K>
hipError_t pack_rows(const u32* rows, u64 n, int arity, int w, K* out, hipStream_t s);
// (c0 << w) | c1  ->  (c1 << w) | c0
template <typename K>
hipError_t swap_cols(const K* in, u64 n, int w, K* out, hipStream_t s);
template <typename K>
hipError_t unpack_rows(const K* keys, u64 n, int arity, int w, u32* rows, hipStream_t s,
                       u32 sub = 0);
// out[0] = lower_bound(keys, lo), out[1] = lower_bound(keys, hi) (device).
template <typename K>
hipError_t key_range(const K* keys, u64 n, K lo, K hi, u64* out, hipStream_t s);

// ---------------------------------------------------------------- join
// Values of the current pair (c0, c1) and of the inner tuple's non-join
// column are numbered 0, 1, 2, and 3 is the constant 0 (the second column
// of a unary relation).  The output pair is (v[src0], v[src1]); a
// filter fa >= 0 keeps it only when v[fa] != v[fb], a filter ea >= 0 only
// when v[ea] == v[eb] (a variable repeated in an atom, or an atom whose two
// variables are both already bound).
struct JoinSpec {
  int outer_col;  // which column of the outer pair is the join key
  int src0, src1;
  int fa, fb;
  int ea, eb;
  int w;   // id bits of a column
  int dd;  // nonzero: drop outputs repeated within a tile (join_expand)
};

// A join (or, with ai == 0, a projection) over relations of arity up to 4
// (wide.hip).  Tuples are packed w bits per column, column 0 most
// significant.  The outer (carried) tuple has ao columns; the inner is an
// index of ai columns whose first nj are the join columns, matched in order
// with outer columns jo[0..nj).  Column sources: 0..3 a column of the
// outer, 4..7 a column of the inner (in the index's column order), 8 the
// constant 0.  The output has nout columns src[0..nout); it is kept when
// every `!=` test (fa[f], fb[f]) and every `==` test (ea[f], eb[f]) holds.
struct WideSpec {
  int w;
  int ao, ai, nj;
  int jo[4];
  int nout;
  int src[4];
  int nf, fa[4], fb[4];
  int ne, ea[4], eb[4];
};

template <typename K>
__host__ __device__ __forceinline__ K wide_src(int s, K ok, K ik, const WideSpec& ws) {
  const K mask = (K(1) << ws.w) - 1;
  if (s < 4) return (ok >> ((ws.ao - 1 - s) * ws.w)) & mask;
  if (s < 8) return (ik >> ((ws.ai - 1 - (s - 4)) * ws.w)) & mask;
  return K(0);
}

template <typename K>
__host__ __device__ __forceinline__ K wide_gather(K ok, K ik, const WideSpec& ws, bool& pass) {
  K v = 0;
  for (int t = 0; t < ws.nout; ++t) v = (v << ws.w) | wide_src(ws.src[t], ok, ik, ws);
  pass = true;
  for (int f = 0; f < ws.nf; ++f)
    pass = pass && wide_src(ws.fa[f], ok, ik, ws) != wide_src(ws.fb[f], ok, ik, ws);
  for (int f = 0; f < ws.ne; ++f)
    pass = pass && wide_src(ws.ea[f], ok, ik, ws) == wide_src(ws.eb[f], ok, ik, ws);
  return v;
}

bool wide_spec_ok(const WideSpec& ws);
// Runs of equal prefix key >> shift (K-wide comparison).
template <typename K>
hipError_t wide_count_runs(const K* keys, u64 n, int shift, u64* d_runs, hipStream_t s);
// Hash index of the runs of equal prefix, keyed by the prefix's fingerprint
// (table of `cap` zeroed slots, cap > runs).
template <typename K>
hipError_t wide_hisa_build(const K* keys, u64 n, int shift, Slot* table, u64 cap, hipStream_t s,
                           LaunchTimer* timer = nullptr);
// (run start, run length) in `inner` (an index of ws.ai columns) of every
// outer tuple's probe value; length 0 when absent.
template <typename K>
hipError_t wide_probe(const K* outer, u64 n, const WideSpec& ws, const Slot* table, u64 cap,
                      const K* inner, u32* start, u32* len, hipStream_t s,
                      LaunchTimer* timer = nullptr);
template <typename K>
hipError_t wide_probe_learned(const K* outer, u64 n, const WideSpec& ws, const LearnedView<K>& lv,
                              u32* start, u32* len, hipStream_t s, LaunchTimer* timer = nullptr);
// A join with no shared column: (0, n_inner) for every outer tuple.
hipError_t wide_probe_all(u64 n, u64 n_inner, u32* start, u32* len, hipStream_t s,
                          LaunchTimer* timer = nullptr);
// The expand of join_expand_tiles (8 outputs per thread) with WideSpec
// outputs and tests.
template <typename K>
hipError_t wide_expand_tiles(const K* outer, u64 n_outer, const u64* off, const u32* start,
                             const K* inner, u64 total, const WideSpec& ws, const u64* parts,
                             u64 tile0, u64 tiles, K* out, u64* cursor, hipStream_t s,
                             LaunchTimer* timer = nullptr);
// One-atom bodies (ai == 0): every input tuple mapped by ws; with tests,
// survivors are appended at *cursor, else output i goes to out[i].
template <typename K>
hipError_t wide_project(const K* in, u64 n, const WideSpec& ws, K* out, u64* cursor,
                        hipStream_t s);
// out[i] = in[i] with columns reordered: column c of the output is column
// perm[c] of the input (a columns).
template <typename K>
hipError_t wide_permute(const K* in, u64 n, int a, int w, const int* perm, K* out,
                        hipStream_t s);
// Row-major n x a uint32 rows to packed keys and back (sub is subtracted
// from every id on the way out).
template <typename K>
hipError_t wide_pack(const u32* rows, u64 n, int a, int w, K* out, hipStream_t s);
template <typename K>
hipError_t wide_unpack(const K* keys, u64 n, int a, int w, u32* rows, hipStream_t s, u32 sub);

template <typename K>
hipError_t join_probe(const K* outer, u64 n, const JoinSpec& js, const Slot* table, u64 cap,
                      u32* start, u32* len, hipStream_t s, LaunchTimer* timer = nullptr);
// The same probe through a learned index of the inner sorted array: the run
// of join key jc is [lower_bound(jc << w), lower_bound((jc + 1) << w)).
template <typename K>
hipError_t join_probe_learned(const K* outer, u64 n, const JoinSpec& js,
                              const LearnedView<K>& lv, u32* start, u32* len, hipStream_t s,
                              LaunchTimer* timer = nullptr);
// The expand gives each thread `items` outputs (4, 8 or 16): tiles of
// 256 * items merged outer tuples and outputs per workgroup.  Every call of
// one join must use the same items.
bool join_items_ok(int items);
u64 join_parts(u64 n_outer, u64 total, int items = 8);  // entries of the partition array
u64 join_tiles(u64 n_outer, u64 total, int items = 8);  // expand tiles (join_parts - 1)
u64 join_tile_outputs(int items = 8);                   // most outputs one tile emits
// Merge-path partition of the expand's tiles (parts: join_parts entries).
hipError_t join_partition(const u64* off, u64 n_outer, u64 total, u64* parts, hipStream_t s,
                          int items = 8);
// Expands tiles tile0 .. tile0 + tiles - 1 only (parts from join_partition).
// Unfiltered outputs go to out[j - j0], j0 the first output index of tile0;
// filtered ones (or with js.dd) are appended at *cursor.
template <typename K>
// An inner kept as two sorted runs: with inner2, entries n_split + i of
// off/start (n_outer = 2 * n_split entries) are the runs of outer tuple i
// in inner2; the outer array then holds n_split tuples.
hipError_t join_expand_tiles(const K* outer, u64 n_outer, const u64* off, const u32* start,
                             const K* inner, u64 total, const JoinSpec& js, const u64* parts,
                             u64 tile0, u64 tiles, K* out, u64* cursor, hipStream_t s,
                             LaunchTimer* timer = nullptr, int items = 8,
                             const K* inner2 = nullptr, u64 n_split = ~u64(0));
// Expands every (outer, inner run) pair.  Without a filter, output j goes
// to out[j]; with one, survivors are appended at *cursor (device, u64).
// With js.dd, an output equal to an earlier output of the same tile (its
// merged outer and output slots) is dropped as well, and the rest are
// appended at *cursor: the result is the same set with fewer duplicates.
template <typename K>
hipError_t join_expand(const K* outer, u64 n_outer, const u64* off, const u32* start,
                       const K* inner, u64 total, const JoinSpec& js, u64* parts, K* out,
                       u64* cursor, hipStream_t s, LaunchTimer* timer = nullptr, int items = 8,
                       const K* inner2 = nullptr, u64 n_split = ~u64(0));
// A rule body of one atom: projects (and filters) every outer pair.
template <typename K>
hipError_t project(const K* in, u64 n, const JoinSpec& js, K* out, u64* cursor, hipStream_t s);

// Nested evaluation of a two-join body (the paper's nested joins, kept as an
// ablation): join q probes inner[q] through table[q] (hash) or lv[q].
template <typename K>
struct NestedJoin {
  const K* inner[2];
  const Slot* table[2];
  u64 cap[2];
  LearnedView<K> lv[2];
  JoinSpec js[2];
};
// With out == null: counts each outer tuple's kept outputs into count[],
// their exclusive prefix into off[] and the total into *d_total (device),
// using scan_ws (scan_workspace_bytes(n)); an outer tuple with 2^32 or more
// outputs sets *too_many (device, zeroed by the caller) and the results
// are void.  With out: writes the outputs of outer tuple i at
// out[off[i]...].
template <typename K>
hipError_t join_nested(const K* outer, u64 n, const NestedJoin<K>& nj, u32* count, u64* off,
                       u64* d_total, u32* too_many, void* scan_ws, K* out, hipStream_t s);

// --------------------------------------------------- fused iteration
// One workgroup runs every rule of the stratum for a small iteration (see
// fused.hip).  Relations are numbered 0 .. nrels-1 (the IDB relations);
// each owns kFusedSlots words of `counts` (device memory):
//   [0] |delta| read this iteration   [1] |full|
//   [2] |new delta| written           [3] distinct new tuples
//   [4] new tuples after filters      [5] join outputs before filters
//   [6] |tail|: a small sorted run of recent deltas kept beside full (full
//       and tail are disjoint; the relation is their union)
// and counts[kFusedOverflow] is set to 1 when the candidates of a head (or
// a first join's result) exceed the LDS capacity; then every [2] is 0 and
// nothing else of the iteration is valid.
constexpr int kFusedThreads = 1024;
constexpr int kFusedMaxRels = 4;
constexpr int kFusedMaxPlans = 4;
constexpr int kFusedMaxSteps = 2;
constexpr int kFusedSlots = 8;
constexpr int kFusedOverflow = kFusedMaxRels * kFusedSlots;
constexpr int kFusedCountWords = kFusedOverflow + 1;

template <typename K>
struct FusedStep {
  const K* inner;       // the inner relation's sorted array
  const Slot* table;    // its hash index, or null: probe through lv
  u64 cap;
  LearnedView<K> lv;
  JoinSpec js;          // dd is ignored
};

template <typename K>
struct FusedPlan {
  int outer;   // relation whose delta is the outer side
  int head;    // relation the outputs go to
  int nsteps;  // 0: a body of one atom, projected by steps[0].js
  FusedStep<K> steps[kFusedMaxSteps];
};

template <typename K>
struct FusedIteration {
  int nrels, nplans, w;
  FusedPlan<K> plans[kFusedMaxPlans];
  const K* delta_in[kFusedMaxRels];
  const K* full[kFusedMaxRels];
  // learned index over full (n == 0: none; used only while n equals the
  // full size in counts), which narrows each membership search to a window
  LearnedView<K> full_lm[kFusedMaxRels];
  const K* tail[kFusedMaxRels];
  K* delta_out[kFusedMaxRels];  // room for cap_b keys each
  u64* counts;                  // kFusedCountWords words
};

// Workgroups of the first phase of a fused iteration: each joins a slice of
// every delta and tests its candidates; one workgroup then deduplicates
// their survivors into the deltas.
constexpr int kFusedGroups = 64;

template <typename K>
struct FusedScratch {
  K* surv;      // [rel][group] runs of cap_c keys: new candidates
  K* pres;      // [rel][group] runs of cap_c keys: candidates already held
  u64* counts;  // [rel][group][4]: |surv|, |pres|, candidates, join outputs
};

// LDS of one phase-A workgroup: cap_c candidate keys (a power of two),
// cap_t keys of a first join's result, and per-thread staging.  The
// finishing workgroup holds cap_b keys (a power of two): the new tuples of
// one relation in one iteration.
template <typename K>
u64 fused_lds_bytes(u32 cap_c, u32 cap_t);
// Device scratch of fused_iteration for nrels relations.
template <typename K>
u64 fused_scratch_bytes(u32 cap_c, int nrels);
// Allows the launches' dynamic LDS sizes (call once before fused_iteration).
template <typename K>
hipError_t fused_prepare(u32 cap_c, u32 cap_t, u32 cap_b);
template <typename K>
hipError_t fused_iteration(const FusedIteration<K>& it, u32 cap_c, u32 cap_t, u32 cap_b,
                           void* scratch, hipStream_t s);
// out = merge(tail, new delta) of relation r, sizes from counts[r][6] and
// counts[r][2]; the grid covers max_out outputs, and `parts` holds
// fused_merge_tiles(max_out) + 1 words.  Nothing runs after an overflow or
// for an empty delta.
u64 fused_merge_tiles(u64 max_out);
template <typename K>
hipError_t fused_merge(const K* tail, const K* delta, const u64* counts, int r, u64 max_out,
                       u64* parts, K* out, hipStream_t s);
// counts[r][6] += counts[r][2]; counts[r][0] = counts[r][2] (no overflow).
hipError_t fused_advance(u64* counts, int nrels, hipStream_t s);

}  // namespace hl
