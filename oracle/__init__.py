"""Oracle: plain CPU implementations that the GPU path is checked against.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code with the GPU library (``paper_2311_02206_amd``) and never imports it.

Contents:
  * ``evaluate``: a single-threaded std::set semi-naive evaluator of positive
    Datalog (Section 2, semi-naive evaluation; Section 5.1, the fixpoint
    workflow), with a naive mode as a second algorithm;
  * ``reach_bfs_histogram`` / ``reach_from``: per-source breadth-first search
    for transitive closure, an independent checker of Reach (Section 1),
    with the per-iteration delta sizes it implies for the linear and for
    the nonlinear (doubling) closure program;
  * ``sg_tree_closed_form``: the same-generation relation of a rooted tree in
    closed form, an independent checker of SG (Section 2);
  * ``reach_verify``, ``reach_verify_many``, ``sg_tree_verify``: whole-relation
    checks of fetched Reach and SG relations at any size, every row
    included (``closure_check.cpp``, threads over sources or instances).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "liboracle.so")
_SOURCES = ("semi_naive.cpp", "closure_check.cpp", "host_sort.cpp")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C++ oracle with g++ into ``oracle/_build/liboracle.so``."""
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread",
                        *[os.path.join(_HERE, f) for f in _SOURCES], "-o", tmp], check=True)
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        newest = max(os.path.getmtime(os.path.join(_HERE, f)) for f in _SOURCES)
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < newest:
            build()
        L = ctypes.CDLL(_SO)
        vp, cp, u64, u32 = ctypes.c_void_p, ctypes.c_char_p, ctypes.c_uint64, ctypes.c_uint32
        L.or_create.restype = vp
        L.or_destroy.argtypes = [vp]
        L.or_error.restype = cp
        L.or_error.argtypes = [vp]
        L.or_declare.argtypes = [vp, cp, ctypes.c_int, ctypes.c_int]
        L.or_load.argtypes = [vp, cp, vp, u64]
        L.or_program.argtypes = [vp, cp]
        L.or_run.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_iterations.argtypes = [vp]
        L.or_seconds.argtypes = [vp]
        L.or_seconds.restype = ctypes.c_double
        L.or_count.argtypes = [vp, cp]
        L.or_count.restype = ctypes.c_int64
        L.or_fetch.argtypes = [vp, cp, vp, u64]
        L.or_delta_counts.argtypes = [vp, cp, vp, ctypes.c_int]
        L.or_new_counts.argtypes = [vp, cp, vp, ctypes.c_int]
        L.or_history.argtypes = [vp, cp, ctypes.c_int, ctypes.c_int, vp, u64]
        L.or_history.restype = ctypes.c_int64
        L.or_reach_bfs.argtypes = [u32, vp, u64, vp, ctypes.c_int, ctypes.c_int]
        L.or_reach_bfs.restype = ctypes.c_int64
        L.or_reach_from.argtypes = [u32, vp, u64, u32, vp, u64]
        L.or_reach_from.restype = ctypes.c_int64
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.or_reach_verify.argtypes = [u32, vp, u64, vp, u64, vp, ctypes.c_int, ctypes.c_int, i64p]
        L.or_reach_verify.restype = ctypes.c_int64
        L.or_reach_verify_many.argtypes = [u32, vp, vp, vp, vp, vp, vp, ctypes.c_int,
                                           ctypes.c_int, i64p]
        L.or_reach_verify_many.restype = ctypes.c_int64
        L.or_sg_tree_verify.argtypes = [u32, vp, u64, vp, u64, ctypes.c_int, i64p]
        L.or_sg_tree_verify.restype = ctypes.c_int64
        L.or_host_sort_u64.argtypes = [vp, vp, u64, ctypes.c_int]
        L.or_host_sort_u64.restype = ctypes.c_double
        L.or_host_merge_u64.argtypes = [vp, u64, vp, u64, vp, ctypes.c_int]
        L.or_host_merge_u64.restype = ctypes.c_double
        L.or_host_alloc_init.argtypes = [u64, ctypes.c_int]
        L.or_host_alloc_init.restype = ctypes.c_double
        _lib = L
    return _lib


@dataclass
class Result:
    relations: dict = field(default_factory=dict)   # name -> (n, arity) uint32, sorted
    deltas: dict = field(default_factory=dict)      # name -> per-iteration |delta|
    news: dict = field(default_factory=dict)        # name -> per-iteration |distinct new|
    delta_history: dict = field(default_factory=dict)  # name -> [array per iteration]
    new_history: dict = field(default_factory=dict)
    iterations: int = 0
    seconds: float = 0.0


def evaluate(program: str, edb: dict, idb: dict, mode: str = "semi_naive",
             plant: int = 0, max_iterations: int = 0, history: bool = False) -> Result:
    """Evaluate ``program`` to its fixpoint.

    ``edb`` maps a relation name to a row-major uint32 array ``(n, arity)``;
    ``idb`` maps a relation name to its arity.  Returns every IDB relation
    sorted lexicographically in declared column order, deduplicated, and the
    per-iteration delta sizes (iteration 0 evaluates the EDB-only rules; the
    last iteration is the empty one).  ``plant`` is a test hook that plants a
    known mistake (see ``or_run`` in semi_naive.cpp); 0 means none.
    ``history`` keeps every iteration's delta and new sets (small inputs).
    """
    L = lib()
    h = L.or_create()
    try:
        def check(rc):
            if rc < 0:
                raise RuntimeError("oracle: " + L.or_error(h).decode())
        for name, rows in edb.items():
            rows = np.ascontiguousarray(rows, dtype=np.uint32)
            arity = rows.shape[1] if rows.ndim == 2 else 1
            check(L.or_declare(h, name.encode(), arity, 1))
            check(L.or_load(h, name.encode(), rows.ctypes.data, rows.shape[0]))
        for name, arity in idb.items():
            check(L.or_declare(h, name.encode(), arity, 0))
        check(L.or_program(h, program.encode()))
        check(L.or_run(h, 0 if mode == "semi_naive" else 1, plant, max_iterations,
                       1 if history else 0))
        res = Result(iterations=L.or_iterations(h), seconds=L.or_seconds(h))
        for name, arity in idb.items():
            n = L.or_count(h, name.encode())
            out = np.empty((n, arity), dtype=np.uint32)
            check(L.or_fetch(h, name.encode(), out.ctypes.data, n))
            res.relations[name] = out
            cnt = np.zeros(res.iterations + 1, dtype=np.uint64)
            k = L.or_delta_counts(h, name.encode(), cnt.ctypes.data, len(cnt))
            res.deltas[name] = [int(x) for x in cnt[:k]]
            k = L.or_new_counts(h, name.encode(), cnt.ctypes.data, len(cnt))
            res.news[name] = [int(x) for x in cnt[:k]]
            if history:
                for which, store in ((0, res.delta_history), (1, res.new_history)):
                    per = []
                    for it in range(res.iterations):
                        buf = np.empty((int(cnt.max()) + 1, arity), dtype=np.uint32)
                        m = L.or_history(h, name.encode(), which, it, buf.ctypes.data,
                                         buf.shape[0])
                        check(m)
                        per.append(buf[:m].copy())
                    store[name] = per
        return res
    finally:
        L.or_destroy(h)


def reach_bfs_histogram(n_nodes: int, edges: np.ndarray, threads: int | None = None,
                        max_dist: int = 1 << 16):
    """Per-source BFS over ``edges``.  Returns ``(total_pairs, hist)`` where
    ``hist[d]`` counts the pairs whose shortest path has ``d`` edges."""
    edges = np.ascontiguousarray(edges, dtype=np.uint32)
    hist = np.zeros(max_dist, dtype=np.uint64)
    threads = _threads(threads)
    total = lib().or_reach_bfs(n_nodes, edges.ctypes.data, edges.shape[0], hist.ctypes.data,
                               max_dist, threads)
    if total < 0:
        raise RuntimeError("reach_bfs: bad input or distance histogram too short")
    last = int(np.nonzero(hist)[0].max()) if total else 0
    return int(total), [int(x) for x in hist[:last + 1]]


def reach_from(n_nodes: int, edges: np.ndarray, source: int) -> np.ndarray:
    """Sorted targets reachable from ``source`` by one or more edges."""
    edges = np.ascontiguousarray(edges, dtype=np.uint32)
    out = np.empty(n_nodes, dtype=np.uint32)
    n = lib().or_reach_from(n_nodes, edges.ctypes.data, edges.shape[0], source,
                            out.ctypes.data, n_nodes)
    if n < 0:
        raise RuntimeError("reach_from: bad input")
    return out[:n].copy()


def reach_deltas_from_histogram(hist) -> list:
    """Per-iteration Reach delta sizes implied by a shortest-distance
    histogram: iteration i derives the pairs at distance exactly i+1, and the
    final iteration is the empty one."""
    return [int(x) for x in hist[1:]] + [0]


def doubling_deltas_from_histogram(hist) -> list:
    """Per-iteration delta sizes of the nonlinear closure
    T(x, y) :- E(x, y).  T(x, y) :- T(x, z), T(z, y).
    under Jacobi semi-naive evaluation, from the shortest-distance
    histogram: iteration 0 holds the pairs at distance 1, and after
    iteration i the relation holds exactly the pairs at distance <= 2^i
    (a path of length in (2^(i-1), 2^i] splits into two paths of length at
    most 2^(i-1), at least one of them longer than 2^(i-2), i.e. new in
    iteration i-1), so iteration i adds distances 2^(i-1)+1 .. 2^i.  The
    final iteration is the empty one."""
    hist = [int(x) for x in hist]
    out = [hist[1] if len(hist) > 1 else 0]
    lo = 2
    while lo < len(hist):
        hi = 2 * (lo - 1)  # distances lo .. hi = 2^(i-1)+1 .. 2^i
        out.append(sum(hist[lo:hi + 1]))
        lo = hi + 1
    return out + [0] if out[-1] else out


def sg_tree_closed_form(edges: np.ndarray):
    """Same generation on a rooted tree, in closed form.

    With Edge = (parent, child) pairs of a rooted tree, SG(x, y) holds iff
    x != y and x, y are at the same depth >= 1.  Rule 1 derives the sibling
    pairs (lowest common ancestor one level up); a pair whose lowest common
    ancestor is k+1 levels up is first derived in iteration k.  Returns
    ``(total, deltas)`` with the trailing empty iteration included.
    """
    edges = np.asarray(edges, dtype=np.int64)
    n = int(edges.max()) + 1 if len(edges) else 1
    parent = np.full(n, -1, dtype=np.int64)
    parent[edges[:, 1]] = edges[:, 0]
    depth = np.zeros(n, dtype=np.int64)
    # ids of a breadth-first tree are not assumed: iterate to a fixpoint
    changed = True
    while changed:
        nd = np.where(parent >= 0, depth[np.maximum(parent, 0)] + 1, 0)
        changed = bool((nd != depth).any())
        depth = nd
    maxd = int(depth.max())
    # anc[j][v] = ancestor of v j levels up (or -1)
    anc = [np.arange(n, dtype=np.int64)]
    for _ in range(maxd):
        prev = anc[-1]
        anc.append(np.where(prev >= 0, parent[np.maximum(prev, 0)], -1))
        anc[-1][prev < 0] = -1
    deltas = [0] * (maxd + 1)
    total = 0
    for d in range(1, maxd + 1):
        nodes = np.nonzero(depth == d)[0]
        nd_ = len(nodes)
        total += nd_ * (nd_ - 1)

        def ordered_pairs_sharing(level):
            a = anc[level][nodes]
            _, c = np.unique(a, return_counts=True)
            return int((c * (c - 1)).sum())
        # pairs whose ancestors k levels up differ but k+1 levels up coincide
        for k in range(0, d):
            same_up = ordered_pairs_sharing(k + 1)
            same_here = ordered_pairs_sharing(k) if k > 0 else 0
            deltas[k] += same_up - same_here
    while deltas and deltas[-1] == 0:
        deltas.pop()
    deltas.append(0)
    return total, deltas


def _threads(threads):
    # at most 16: the share of host cores that goes with one GPU
    return int(threads or max(1, min(16, os.cpu_count() or 1)))


def reach_verify(n_nodes: int, edges: np.ndarray, rows: np.ndarray, threads: int | None = None,
                 max_dist: int = 1 << 16):
    """Whole-relation check of a fetched Reach relation: for every source, a
    breadth-first search over ``edges`` must mark exactly that source's rows
    (strictly increasing, all marked, as many as marked nodes).  Returns
    ``(mismatching_sources, first_bad_source, hist)`` with ``hist[d]`` the
    number of pairs at shortest distance ``d``; raises on unsorted rows or
    ids out of range."""
    edges = np.ascontiguousarray(edges, dtype=np.uint32)
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    hist = np.zeros(max_dist, dtype=np.uint64)
    bad = ctypes.c_int64(-1)
    r = lib().or_reach_verify(n_nodes, edges.ctypes.data, edges.shape[0],
                              rows.ctypes.data if len(rows) else None, rows.shape[0],
                              hist.ctypes.data, max_dist, _threads(threads), ctypes.byref(bad))
    if r == -1:
        raise ValueError("reach_verify: rows not strictly increasing or ids out of range")
    if r == -2:
        raise ValueError("reach_verify: a distance exceeds max_dist")
    last = int(np.nonzero(hist)[0].max()) if hist.any() else 0
    return int(r), int(bad.value), [int(x) for x in hist[:last + 1]]


def reach_verify_many(nodes, edges_list, rows_list, threads: int | None = None,
                      max_dist: int = 1 << 12):
    """``reach_verify`` over independent instances (instance-local ids).
    Returns ``(mismatching_instances, first_bad_instance, summed_hist)``."""
    k = len(nodes)
    nodes = np.ascontiguousarray(nodes, dtype=np.uint32)
    e_off = np.zeros(k + 1, dtype=np.uint64)
    e_off[1:] = np.cumsum([len(x) for x in edges_list])
    r_off = np.zeros(k + 1, dtype=np.uint64)
    r_off[1:] = np.cumsum([len(x) for x in rows_list])
    E = np.ascontiguousarray(np.concatenate([np.asarray(x, np.uint32).reshape(-1, 2)
                                             for x in edges_list]) if k else
                             np.zeros((0, 2), np.uint32))
    R = np.ascontiguousarray(np.concatenate([np.asarray(x, np.uint32).reshape(-1, 2)
                                             for x in rows_list]) if k else
                             np.zeros((0, 2), np.uint32))
    hist = np.zeros(max_dist, dtype=np.uint64)
    bad = ctypes.c_int64(-1)
    r = lib().or_reach_verify_many(k, nodes.ctypes.data, e_off.ctypes.data,
                                   E.ctypes.data if len(E) else None, r_off.ctypes.data,
                                   R.ctypes.data if len(R) else None, hist.ctypes.data,
                                   max_dist, _threads(threads), ctypes.byref(bad))
    if r == -1:
        raise ValueError("reach_verify_many: rows not strictly increasing or ids out of range")
    if r == -2:
        raise ValueError("reach_verify_many: a distance exceeds max_dist")
    last = int(np.nonzero(hist)[0].max()) if hist.any() else 0
    return int(r), int(bad.value), [int(x) for x in hist[:last + 1]]


def sg_tree_verify(edges: np.ndarray, rows: np.ndarray, threads: int | None = None):
    """Whole-relation check of a fetched SG relation over a rooted tree
    (Edge = (parent, child)): rows strictly increasing, every row a pair of
    distinct nodes of equal depth >= 1.  With the closed-form count this is
    set equality.  Returns ``(bad_rows, first_bad_row)``."""
    edges = np.ascontiguousarray(edges, dtype=np.uint32)
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    n = int(edges.max()) + 1 if len(edges) else 1
    bad = ctypes.c_int64(-1)
    r = lib().or_sg_tree_verify(n, edges.ctypes.data, edges.shape[0],
                                rows.ctypes.data if len(rows) else None, rows.shape[0],
                                _threads(threads), ctypes.byref(bad))
    if r == -1:
        raise ValueError("sg_tree_verify: rows not strictly increasing or ids out of range")
    if r == -3:
        raise ValueError("sg_tree_verify: the edges are not a rooted tree")
    return int(r), int(bad.value)


def host_sort_u64(keys: np.ndarray, threads: int | None = None) -> float:
    """Sorts a uint64 array in place on ``threads`` host threads (the host
    side of the sort/merge/memory microbenchmark); returns the seconds."""
    assert keys.dtype == np.uint64 and keys.flags.c_contiguous
    tmp = np.empty_like(keys)
    return lib().or_host_sort_u64(keys.ctypes.data, tmp.ctypes.data, keys.size,
                                  _threads(threads))


def host_merge_u64(a: np.ndarray, b: np.ndarray, out: np.ndarray,
                   threads: int | None = None) -> float:
    """out = merge of ascending uint64 arrays a and b on host threads;
    returns the seconds."""
    assert a.dtype == b.dtype == out.dtype == np.uint64 and out.size == a.size + b.size
    return lib().or_host_merge_u64(a.ctypes.data, a.size, b.ctypes.data, b.size,
                                   out.ctypes.data, _threads(threads))


def host_alloc_init(nbytes: int, threads: int | None = None) -> float:
    """Seconds to allocate a fresh host buffer of nbytes and write every
    byte once on host threads."""
    s = lib().or_host_alloc_init(nbytes, _threads(threads))
    if s < 0:
        raise MemoryError(f"host allocation of {nbytes} bytes failed")
    return s
