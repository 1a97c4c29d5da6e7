/*
 * hisalog: semi-naive Datalog fixpoint evaluation on one AMD MI355X (gfx950)
 * over hash-indexed sorted arrays (HISA).
 *
 * The method is that of "Optimizing Datalog for the GPU" (Sun, Shovon,
 * Gilray, Kumar, Micinski): relations are sorted arrays of packed tuples
 * with an open-addressing hash index from join key to run start (Section 4);
 * each fixpoint iteration joins the delta of each recursive relation against
 * the indexed full relations (Section 5.1, Algorithm 3), deduplicates the new
 * tuples by sorting (Section 4.2), subtracts full to form the next delta
 * (Section 5.1, "Populating delta") and merges delta into full (Section 5.1,
 * "Merging Full with Delta"), with multi-atom bodies evaluated as a chain of
 * materialised binary joins (Section 5.2) and merge buffers kept and grown
 * eagerly (Section 5.3).  Evaluation stops when every delta is empty.
 *
 * Conventions for every call:
 *   - Return value: HL_OK (0) or a negative HL_E_* code; no call aborts or
 *     throws.  hl_last_error(engine) describes the most recent failure.
 *   - Relation tuples are uint32 columns; host and device row buffers are
 *     row-major n x arity.  Arity 1 and 2 are supported (a unary tuple is
 *     stored as the pair (x, 0)); other arities are rejected with
 *     HL_E_UNSUPPORTED.
 *   - One engine is used by one host thread at a time.  Device work is
 *     enqueued on the engine's stream; calls that return host-visible
 *     results synchronise that stream before returning.
 *   - Pointers named d_* are device pointers (HIP device memory of the
 *     engine's device); all others are host pointers.  The caller keeps
 *     ownership of every buffer it passes in.
 */
#ifndef HISALOG_H
#define HISALOG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define HL_OK 0
#define HL_E_INVALID (-1)     /* bad argument, unknown relation, parse error */
#define HL_E_NOMEM (-2)       /* device memory (arena or budget) exhausted */
#define HL_E_DEVICE (-3)      /* a HIP runtime call failed; text in hl_last_error */
#define HL_E_STATE (-4)       /* call not allowed in the engine's current state */
#define HL_E_CAPACITY (-5)    /* caller's output buffer too small; size returned */
#define HL_E_UNSUPPORTED (-6) /* a valid program or option this build does not run */

/* ---------------------------------------------------------------- flags */
#define HL_FLAG_NO_EBM 0x1u /* disable eager buffer management (exact-size
                               buffers, reallocated on every growth, and
                               every released block returned with hipFree:
                               the paper's "Normal" column of Table 1) */
#define HL_FLAG_KERNEL_TIMING 0x2u /* time every launch of the kernels listed
                                      under hl_kernel_stats with HIP events */
#define HL_FLAG_LEARNED_INDEX 0x4u /* probe inner relations and test membership
                                      in full through a learned position index
                                      (see hl_learned_query) instead of the HISA
                                      hash; results are identical */
#define HL_FLAG_JOIN_DEDUP 0x8u /* drop repeated join outputs inside an
                                   expand tile: while a head relation's joins
                                   produced at least 1.5 outputs per distinct
                                   new tuple in the previous iteration (and in
                                   the first one), the last join of each of
                                   its rules groups its outer by the column
                                   carried to the head and drops repeats
                                   within each tile in LDS.  Results are
                                   identical; fewer keys are sorted, at the
                                   price of a slower expand (measured a net
                                   loss at 2,048-slot tiles, hence off by
                                   default) */
#define HL_FLAG_FUSED 0x10u /* run small iterations of the recursive stratum
                               as one fused launch: a single workgroup joins
                               every delta with its inner indexes, sorts,
                               deduplicates and subtracts full in LDS, and a
                               merge reads its sizes from device memory, so
                               an iteration costs a few launches and one
                               synchronisation instead of dozens of each.
                               Applies when every join inner is an EDB
                               relation (Reach, same-generation and the
                               like; at most 4 IDB relations, 4 rule
                               variants, 2 joins per rule), eager buffer
                               management is on, and the last iteration's
                               output rate predicts that the candidates fit
                               in LDS (see fused_capacity); an iteration
                               whose candidates do not fit is rerun on the
                               multi-kernel path.  Results are identical */
#define HL_FLAG_HIP_GRAPH 0x20u /* HL_FLAG_FUSED, with each fused iteration
                                   (its launches and the copy of its counts
                                   to the host) captured once in a HIP graph
                                   and replayed while its buffers and grid
                                   stay the same */
#define HL_FLAG_NESTED_JOINS 0x40u /* ablation of Section 5.2: evaluate a rule
                                     body of two joins as nested loops, one
                                     thread per outer tuple walking both
                                     runs, instead of materialising the first
                                     join's result and joining it again
                                     (load-balanced).  Results are identical;
                                     `join_outputs` then counts the kept
                                     outputs.  Bodies whose outputs exceed one
                                     sort chunk keep the materialised form */

#define HL_FLAG_NO_LEVELS 0x80u /* keep every relation probed as a join inner
                                  as one sorted array, its indexes rebuilt
                                  (or refitted) after every merge, instead
                                  of two levels: full with its indexes plus
                                  a short tail run with indexes of its own,
                                  which joins probe both of and whose
                                  deltas leave full and its indexes
                                  untouched until the tail is folded in (the
                                  merge-cost problem of Section 6.5).
                                  Results are identical */

/* Kernels reported by hl_kernel_stats. */
#define HL_KERNEL_RADIX_HIST 0    /* digit histogram of one radix pass */
#define HL_KERNEL_RADIX_SCATTER 1 /* stable scatter of one radix pass */
#define HL_KERNEL_UNIQUE_DIFF 2   /* dedup + membership test against full */
#define HL_KERNEL_MERGE 3         /* merge path of full and delta */
#define HL_KERNEL_JOIN_PROBE 4    /* hash probe of every outer tuple */
#define HL_KERNEL_JOIN_EXPAND 5   /* load-balanced expansion of the runs */
#define HL_KERNEL_HISA_BUILD 6    /* hash index insertion */
#define HL_KERNEL_LEARNED_FIT 7   /* learned index refit (table + error bounds) */
#define HL_KERNEL_COUNT 8

/* Phases of one fixpoint, timed with HIP events (milliseconds). */
#define HL_PHASE_INDEX_EDB 0 /* EDB dedup + HISA builds before iteration 0 */
#define HL_PHASE_JOIN 1      /* probes and expands of every rule */
#define HL_PHASE_SORT 2      /* radix sort of the new tuples */
#define HL_PHASE_DIFF 3      /* dedup + subtraction of full (delta) */
#define HL_PHASE_MERGE 4     /* full := full U delta */
#define HL_PHASE_INDEX 5     /* index refresh of probed full relations */
#define HL_PHASE_FUSED 6     /* fused iterations (HL_FLAG_FUSED), all steps */
#define HL_PHASE_COUNT 7

typedef struct hl_engine hl_engine;

typedef struct hl_options {
  int32_t device;            /* HIP device ordinal */
  uint32_t flags;            /* HL_FLAG_* */
  void* arena;               /* optional caller-owned device memory that all
                                engine buffers are carved from (never freed
                                by the engine); NULL: the engine allocates
                                with hipMalloc up to hbm_budget_bytes */
  uint64_t arena_bytes;      /* size of arena */
  uint64_t hbm_budget_bytes; /* cap on the device memory the engine holds
                                when arena == NULL: live buffers plus the
                                released blocks it keeps for reuse (the
                                latter are returned first when the cap or
                                the device would be exceeded; 0: no cap
                                beyond the device) */
  void* stream;              /* hipStream_t to enqueue on; NULL: own stream */
  float ebm_k;               /* growth factor k of Section 5.3: a buffer that
                                must grow to hold |full| + |delta| is
                                reallocated to |full| + k |delta| (default 8) */
  float hash_load_factor;    /* HISA hash table load factor in (0, 1]
                                (default 0.5; Section 6.4 uses 0.8, which
                                costs ~13 slot reads per linear-probing miss
                                against ~2.5 at 0.5) */
  uint32_t sort_chunk_log2;  /* an iteration's new tuples are sorted in chunks
                                of at most 2^sort_chunk_log2 keys (12..31;
                                0: just under 2^32 keys for 4-byte keys,
                                2^31 for 8-byte keys) */
  uint32_t fused_capacity;   /* new tuples (distinct candidates, new or
                                already held) a fused iteration gathers per
                                relation in LDS (HL_FLAG_FUSED): a power of
                                two from 1,024 up to what one workgroup's
                                LDS holds; 0: the largest that fits (16,384
                                64-bit or 32,768 32-bit keys on a 160 KB-LDS
                                device).  Larger is not faster per
                                iteration; it lets more iterations fuse */
  uint32_t expand_tile;      /* join outputs (and merged outer tuples) one
                                expand workgroup handles: 1024, 2048 or
                                4096 (0: 2048); hl_autotune measures all
                                three */
  uint32_t sort_tile;        /* keys per radix sort tile: 4096 or 8192 (0:
                                8192); hl_autotune measures both */
  uint32_t diff_tile;        /* sorted candidates per set difference tile:
                                2048 or 4096 (0: 4096); hl_autotune
                                measures both */
  uint32_t outer_slice_log2; /* a join's outer side is taken at most
                                2^outer_slice_log2 tuples at a time
                                (8..31; 0: 28), which bounds the join's
                                scratch (16 bytes per outer tuple) and a
                                multi-atom rule's intermediate result */
  uint64_t tail_min_bytes;   /* a relation's new tuples go to a sorted tail
                                run beside its full relation (folded in when
                                the tail passes an eighth of full) once full
                                holds this many bytes (0: 64 MiB); for a
                                relation probed as a join inner the tail
                                has indexes of its own (see
                                HL_FLAG_NO_LEVELS).  Results are identical */
} hl_options;

typedef struct hl_stats {
  uint32_t iterations;           /* iterations run, including iteration 0 (the
                                    EDB-only rules) and the final empty one */
  uint32_t key_bytes;            /* 4 or 8: packed key width chosen at run */
  uint32_t id_bits;              /* w: bits per column in a packed key */
  uint32_t fused_iterations;     /* iterations run by the fused launch
                                    (HL_FLAG_FUSED) */
  uint64_t idb_tuples;           /* sum over IDB relations of |full| at fixpoint */
  uint64_t candidates;           /* new tuples written for sorting over all
                                    iterations (join outputs after filters
                                    and in-tile dedup) */
  uint64_t peak_bytes;           /* peak device bytes held by the engine */
  uint64_t allocations;          /* hipMalloc calls made during the run (blocks
                                    reused from the engine's own released
                                    blocks are not counted) */
  uint64_t ebm_reuses;           /* buffer requests served without allocating */
  double seconds;                /* wall time of hl_run (host clock) */
  double phase_ms[HL_PHASE_COUNT];
  uint64_t join_outputs;         /* outputs of the joins (and one-atom rules)
                                    whose results go to a head relation,
                                    before filters and in-tile dedup;
                                    `candidates` counts those kept */
  uint32_t fused_overflows;      /* fused launches whose candidates did not
                                    fit (each such iteration was rerun on the
                                    multi-kernel path) */
  uint32_t graph_captures;       /* HIP graphs captured (HL_FLAG_HIP_GRAPH);
                                    the other fused iterations replayed one */
} hl_stats;

/* Fills *opt with defaults: device 0, no arena, own stream, ebm_k 8,
 * load factor 0.5. */
int hl_options_init(hl_options* opt);

/* Creates an engine on opt->device.  *out receives the handle (NULL on
 * failure).  With opt->stream set, the engine never creates or destroys a
 * stream; the caller keeps that stream alive until hl_destroy.
 * opt->device == -1 creates a planning-only engine that touches no device:
 * hl_declare, hl_index and hl_program work (so programs can be checked),
 * loads, runs and primitives return HL_E_STATE. */
int hl_create(const hl_options* opt, hl_engine** out);

/* Releases every device buffer the engine allocated (never the caller's
 * arena or stream).  NULL is ignored. */
void hl_destroy(hl_engine* e);

/* Declares relation `name` (identifier, at most 63 bytes) of `arity` columns
 * (1 to 4; others HL_E_UNSUPPORTED), extensional (is_edb != 0: loaded with
 * hl_load*) or intensional (derived by rules).  Before hl_program.
 * Duplicate names: HL_E_INVALID. */
int hl_declare(hl_engine* e, const char* name, uint32_t arity, int32_t is_edb);

/* Appends n_rows host rows (row-major n x arity uint32) to EDB relation
 * `name`.  The rows are copied before the call returns.  Duplicates are
 * removed at hl_run (relations are sets).  Any uint32 value is a legal id. */
int hl_load(hl_engine* e, const char* name, const uint32_t* rows, uint64_t n_rows);

/* Same from device memory d_rows (stream-ordered on the engine's stream:
 * d_rows may be reused once the engine's stream has passed this call). */
int hl_load_device(hl_engine* e, const char* name, const uint32_t* d_rows, uint64_t n_rows);

/* Batches of independent instances of one program (an addition to the
 * paper, whose engine runs one database at a time).  Instance k uses ids
 * [0, id_range[k]); the engine maps them to the private range
 * [base_k, base_k + id_range[k]) of one id space (dictionary encoding,
 * base_k = sum of the earlier ranges, total below 2^32), and one fixpoint
 * over the union then computes every instance's own fixpoint in one set
 * of launches per iteration.  This is exact for every program hl_program
 * accepts: joins match equal values only and every rule body is connected,
 * so no derivation mixes instances.  Per-iteration counts (hl_iteration_
 * counts) are totals over the batch.  Call once, before any load. */
int hl_batch_layout(hl_engine* e, const uint32_t* id_range, uint32_t n_inst);

/* Loads EDB rows of every instance: rows[inst_offsets[k] .. inst_offsets[k+1])
 * (row indices; n_inst + 1 offsets, starting at 0) are instance k's rows, with
 * instance-local ids (each must be < id_range[k]: HL_E_INVALID otherwise).
 * The rows are copied before the call returns. */
int hl_load_batched(hl_engine* e, const char* name, const uint32_t* rows,
                    const uint64_t* inst_offsets);

/* Size of instance `inst`'s part of relation `name` after hl_run. */
int hl_batch_count(hl_engine* e, const char* name, uint32_t inst, uint64_t* n);

/* Instance `inst`'s part of relation `name`, sorted, with instance-local ids,
 * into host buffer rows (cap_rows rows); HL_E_CAPACITY and the needed size
 * as for hl_fetch. */
int hl_fetch_batched(hl_engine* e, const char* name, uint32_t inst, uint32_t* rows,
                     uint64_t cap_rows, uint64_t* n_rows);

/* Requests a HISA on relation `name` keyed by its column cols[0]
 * (Section 4: sorted array + hash index).  Only ncols == 1 is supported.
 * Optional: hl_program declares every index its rules probe. */
int hl_index(hl_engine* e, const char* name, const uint32_t* cols, uint32_t ncols);

/* Adds the rules of `text`:  Head(x, y) :- A(x, z), B(z, y), x != y.
 * Positive rules over declared relations; variables are identifiers, `_`
 * is a wildcard in body atoms; `x != y` filters two body variables; `//`
 * and `#` start comments.  Every head variable must occur in the body.
 * A rule body is evaluated as a chain of binary joins (Section 5.2).  A
 * program whose relations are unary or binary and whose every rule is a
 * chain in which each further atom shares one variable with the pair
 * carried so far runs on keys of two columns; any other program (a relation
 * of arity 3-4, a join on two columns, three or four variables live between
 * joins, a cross product: an atom sharing no variable, whose relation is
 * then scanned whole per carried tuple) runs as wide plans.  More than four
 * variables live between joins, or more than four filters or equality
 * tests at one join, give HL_E_UNSUPPORTED. */
int hl_program(hl_engine* e, const char* text);

/* Runs semi-naive evaluation to the fixpoint (Section 5.1), Jacobi order:
 * iteration 0 evaluates the rules whose bodies are EDB-only; iteration
 * i >= 1 evaluates every rule with an IDB body atom once per such atom,
 * that atom over the delta of iteration i-1 and the other IDB atoms over
 * full; deltas are formed and merged after all rules.  Blocking.  May be
 * called again: IDB relations restart from empty.  stats may be NULL. */
int hl_run(hl_engine* e, hl_stats* stats);

/* Settings chosen by hl_autotune. */
typedef struct hl_tuning {
  float hash_load_factor;  /* load factor of the HISA hash tables */
  float ebm_k;             /* eager buffer growth factor */
  uint32_t flags;          /* the chosen HL_FLAG_LEARNED_INDEX,
                              HL_FLAG_JOIN_DEDUP, HL_FLAG_NESTED_JOINS,
                              HL_FLAG_FUSED and HL_FLAG_HIP_GRAPH bits */
  uint32_t trials;         /* settings timed (failed ones included) */
  double best_seconds;     /* fixpoint time under the chosen setting */
  double first_seconds;    /* fixpoint time under the engine's settings
                              before tuning */
  uint32_t expand_tile;    /* the chosen hl_options.expand_tile */
  uint32_t sort_tile;      /* the chosen hl_options.sort_tile */
  uint32_t diff_tile;      /* the chosen hl_options.diff_tile */
  uint32_t reserved;
} hl_tuning;

/* Tunes the engine for the loaded program and data by measurement.  The
 * settings are searched one dimension at a time, starting from the
 * engine's own: how join inners are probed (HISA hash at load factor 0.5,
 * at 0.8, or the learned position index), the join expand tile (1024,
 * 2048 or 4096 outputs per workgroup), the radix sort tile (4096 or 8192
 * keys), the set difference tile (2048 or 4096 candidates), the eager
 * buffer growth factor
 * (1.5 or 8), in-tile dedup of join outputs (off or on), nested
 * evaluation of two-join bodies (off or on, where a rule has one) and,
 * where the recursive rules qualify, fused small iterations (off, on, or
 * on and replayed from HIP graphs).  Each setting
 * runs the fixpoint once to warm up and then `reps` times (at least 1),
 * and is scored by its fastest hl_run time; a setting that runs out of
 * device memory is skipped.  Every setting must give the same per-iteration
 * delta sizes (HL_E_STATE otherwise: results never depend on these
 * settings).  The fastest stays in force for later hl_run calls, and a
 * final run under it leaves the relations computed.  out may be NULL. */
int hl_autotune(hl_engine* e, uint32_t reps, hl_tuning* out);

/* *n = number of tuples of relation `name` (after hl_run). */
int hl_count(hl_engine* e, const char* name, uint64_t* n);

/* Copies relation `name` as sorted (lexicographic in declared column
 * order), duplicate-free row-major uint32 rows into host buffer rows of
 * cap_rows rows.  *n_rows receives the relation size; when cap_rows is
 * smaller the call copies nothing and returns HL_E_CAPACITY. */
int hl_fetch(hl_engine* e, const char* name, uint32_t* rows, uint64_t cap_rows,
             uint64_t* n_rows);

/* Same into device memory d_rows (synchronises before returning). */
int hl_fetch_device(hl_engine* e, const char* name, uint32_t* d_rows, uint64_t cap_rows,
                    uint64_t* n_rows);

/* Per-iteration delta sizes of relation `name` from the last hl_run:
 * counts[i] = |delta| of iteration i, for i < min(cap, iterations);
 * *n_iters = iterations.  which = 0: delta sizes; 1: number of distinct
 * tuples derived in the iteration before subtracting full. */
int hl_iteration_counts(hl_engine* e, const char* name, int32_t which, uint64_t* counts,
                        uint32_t cap, uint32_t* n_iters);

/* With HL_FLAG_KERNEL_TIMING: totals over the last hl_run for kernel
 * `kernel` (HL_KERNEL_*): number of launches, summed launch time in
 * milliseconds (HIP events recorded on the engine's stream right before and
 * after each launch) and summed algorithmic bytes (the bytes the kernel
 * must read and write by definition: inputs once, outputs once).  Without
 * the flag every total is 0. */
int hl_kernel_stats(hl_engine* e, int32_t kernel, uint64_t* launches, double* ms,
                    uint64_t* algorithmic_bytes);

/* Join outputs of rule `rule` (0-based, in program text order) over the
 * last hl_run: *join_outputs = outputs of the rule's last join (its
 * candidates before `!=` filters and dedup; for a one-atom body, its outer
 * tuples), summed over iterations and over the rule's delta variants (one
 * per IDB body atom, Section 5.1); *intermediate = outputs of its earlier
 * joins (the temporarily materialised results of Section 5.2).  Fused
 * iterations (HL_FLAG_FUSED) are not counted here.  HL_E_INVALID for a rule
 * index beyond the program, HL_E_STATE before hl_run. */
int hl_rule_stats(hl_engine* e, uint32_t rule, uint64_t* join_outputs, uint64_t* intermediate);

/* Text of the most recent error of e (never NULL; "" when none). */
const char* hl_last_error(hl_engine* e);

/* Static text for a return code. */
const char* hl_strerror(int code);

/* ------------------------------------------------------------ primitives
 * The kernels of one iteration, exposed on device buffers so each can be
 * checked on its own.  They run on the engine's stream, use its memory
 * (arena or budget) for temporaries and synchronise before returning.
 * key_bytes is 4 (uint32 keys) or 8 (uint64 keys).  Sizes are element
 * counts. */

/* Sorts n keys of d_keys ascending in place by their low `bits` bits
 * (all bits when bits == 0); higher bits must be zero (Section 4.2,
 * Algorithm 1: LSD order over the packed columns).  n < 2^32. */
int hl_sort_keys(hl_engine* e, void* d_keys, uint64_t n, uint32_t key_bytes, uint32_t bits);

/* hl_sort_keys without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The sort's second buffer and its
 * count matrices live in a static device array of 64 MiB that each GPU the
 * library runs on holds until the process ends; the call makes no
 * hipMalloc, hipFree or other allocating call (a copy back into d_keys
 * when the result ends in the scratch copy is a device-to-device copy).
 * Same arguments, order and result as hl_sort_keys; n keys must fit the
 * scratch with their count matrices: about 15.7 million 4-byte or 8.1
 * million 8-byte keys (HL_E_CAPACITY beyond, with the sizes in
 * hl_last_error).  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (from several threads or engines) race; calls
 * made one after another do not, since each synchronises the engine's
 * stream before returning.  Nothing in the array needs to start at zero:
 * every count a pass reads was written by that pass. */
int hl_sort_keys_noalloc(hl_engine* e, void* d_keys, uint64_t n, uint32_t key_bytes,
                         uint32_t bits);

/* d_out = unique(d_sorted) minus d_full (Section 5.1, "Populating delta";
 * Section 4.2, "Deduplication").  d_sorted: n ascending keys (repeats
 * allowed); d_full: n_full ascending distinct keys; d_out: room for n keys.
 * *n_out = |d_out|, *n_unique = distinct keys of d_sorted.  n < 2^32.
 * When n_full <= n the two arrays are walked together in merge-path tiles;
 * otherwise each tile of candidates searches the slice of d_full it spans
 * (the result is the same). */
int hl_unique_diff(hl_engine* e, const void* d_sorted, uint64_t n, const void* d_full,
                   uint64_t n_full, void* d_out, uint64_t* n_out, uint64_t* n_unique,
                   uint32_t key_bytes);

/* d_out (room for na + nb keys) = merge of ascending d_a and d_b
 * (Section 4.2, "Merge operation": merge path). */
int hl_merge(hl_engine* e, const void* d_a, uint64_t na, const void* d_b, uint64_t nb,
             void* d_out, uint32_t key_bytes);

/* Builds a HISA over n ascending keys d_keys whose join column is
 * key >> shift (Section 4.3, Algorithm 2), then answers nq range queries:
 * for join value d_queries[i], d_start[i] = position of the first key with
 * that join value and d_len[i] = number of such keys (0 when absent;
 * d_start is then 0).  *n_runs receives the number of distinct join values.
 * n < 2^32. */
int hl_hisa_query(hl_engine* e, const void* d_keys, uint64_t n, uint32_t key_bytes,
                  uint32_t shift, const uint32_t* d_queries, uint64_t nq, uint64_t* d_start,
                  uint32_t* d_len, uint64_t* n_runs);

/* Learned position index (an addition to the paper's HISA, used by
 * HL_FLAG_LEARNED_INDEX): fits a radix table over the top bits of n
 * ascending keys d_keys (whose values are below 2^key_bits) with an fp32
 * linear model per radix bucket and the bucket's exact error bound, then
 * writes d_pos[i] = lower_bound(d_keys, d_queries[i]) (the first position
 * whose key is >= the query; n if none) for nq queries of the key type.
 * The answer is exact for any query below 2^key_bits: the radix table
 * brackets it and the bound limits the window a binary search scans.
 * n < 2^32. */
int hl_learned_query(hl_engine* e, const void* d_keys, uint64_t n, uint32_t key_bytes,
                     uint32_t key_bits, const void* d_queries, uint64_t nq, uint32_t* d_pos);

#ifdef __cplusplus
}
#endif

#endif /* HISALOG_H */
