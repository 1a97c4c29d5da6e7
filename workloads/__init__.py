"""Seeded synthetic input generators.

This module is shared by the oracle side (tests, CPU baseline) and the GPU
side (tests, bench, smoke).  It holds no Datalog arithmetic at all: it only
turns a seed into EDB relations (uint32 row-major ``(n, 2)`` numpy arrays)
whose shape stands in for the paper's workloads (graphs from SNAP,
SuiteSparse and road networks for Reach / same-generation, Graspan
points-to facts for CSPA; Section 6.2).  None of those datasets is
reproduced here; every relation is drawn from the generators below.

Random numbers come from one counter-based generator: value ``i`` of the
stream with key ``k`` is ``splitmix64(k + (i + 1) * 0x9E3779B97F4A7C15)``
(Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014; the finaliser constants are Vigna's published splitmix64).
Bounded integers use the multiply-shift reduction of the top 32 bits
(Lemire, "Fast random integer generation in an interval", 2019, without the
rejection step: a bias below 2^-32 * n is irrelevant for synthetic inputs),
doubles use the top 53 bits.
"""

from __future__ import annotations

import math

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def splitmix64_scalar(x: int) -> int:
    """One splitmix64 output for state ``x`` (used to derive sub-keys)."""
    z = (x + 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def subkey(seed: int, tag: int) -> int:
    """Key of an independent stream derived from ``seed`` and a small tag."""
    return splitmix64_scalar((seed * 0x100000001B3 + tag) & _MASK64)


def stream_u64(key: int, start: int, count: int) -> np.ndarray:
    """Values ``start .. start+count-1`` of the stream with key ``key``."""
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
        z = np.uint64(key) + idx * _GAMMA
        return _mix(z)


def bounded_u32(u: np.ndarray, n: int) -> np.ndarray:
    """Map uint64 draws to integers in ``[0, n)`` (n <= 2^32)."""
    if not 0 < n <= 1 << 32:
        raise ValueError("bound out of range")
    hi = (u >> np.uint64(32)).astype(np.uint64)
    return ((hi * np.uint64(n)) >> np.uint64(32)).astype(np.uint32)


def unit_double(u: np.ndarray) -> np.ndarray:
    """Map uint64 draws to doubles in ``[0, 1)``."""
    return (u >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def _first_distinct_pairs(draw, m: int, batch: int) -> np.ndarray:
    """First ``m`` distinct pairs with ``u != v`` of the draw stream.

    ``draw(start, count)`` returns the pairs at stream positions
    ``start .. start+count-1``.  The result equals sequential rejection of
    self-loops and repeats, in stream order.
    """
    taken = np.empty(0, dtype=np.uint64)
    parts_u, parts_v = [], []
    start = 0
    have = 0
    while have < m:
        u, v = draw(start, batch)
        start += batch
        keep = u != v
        u, v = u[keep], v[keep]
        key = (u.astype(np.uint64) << np.uint64(32)) | v.astype(np.uint64)
        _, first = np.unique(key, return_index=True)
        first.sort()
        u, v, key = u[first], v[first], key[first]
        fresh = ~np.isin(key, taken, assume_unique=True)
        u, v, key = u[fresh], v[fresh], key[fresh]
        need = m - have
        u, v, key = u[:need], v[:need], key[:need]
        parts_u.append(u)
        parts_v.append(v)
        taken = np.concatenate([taken, key])
        have += len(u)
        if start > 64 * max(m, 1024):
            raise ValueError("cannot draw that many distinct pairs")
    out = np.empty((m, 2), dtype=np.uint32)
    if m:
        out[:, 0] = np.concatenate(parts_u)
        out[:, 1] = np.concatenate(parts_v)
    return out


def erdos_renyi(n_nodes: int, n_edges: int, seed: int) -> np.ndarray:
    """Directed G(n, m): ``n_edges`` distinct non-self pairs, uniform."""
    if n_edges > n_nodes * (n_nodes - 1):
        raise ValueError("too many edges for the node count")
    ku, kv = subkey(seed, 1), subkey(seed, 2)

    def draw(start, count):
        return (bounded_u32(stream_u64(ku, start, count), n_nodes),
                bounded_u32(stream_u64(kv, start, count), n_nodes))

    return _first_distinct_pairs(draw, n_edges, max(2 * n_edges, 1024))


def rmat(scale: int, n_edges: int, seed: int,
         a: float = 0.57, b: float = 0.19, c: float = 0.19) -> np.ndarray:
    """Directed R-MAT graph on ``2^scale`` nodes (Chakrabarti et al. 2004).

    Per edge, ``scale`` levels pick a quadrant MSB-first: (0,0) with
    probability a, (0,1) with b, (1,0) with c, (1,1) with 1-a-b-c.  No noise
    and no label permutation.  Self-loops and repeats are rejected.
    """
    key = subkey(seed, 3)
    ab, abc = a + b, a + b + c

    def draw(start, count):
        u = np.zeros(count, dtype=np.uint32)
        v = np.zeros(count, dtype=np.uint32)
        raw = stream_u64(key, start * scale, count * scale).reshape(count, scale)
        r = unit_double(raw)
        for lvl in range(scale):
            x = r[:, lvl]
            row = (x >= ab).astype(np.uint32)
            col = (((x >= a) & (x < ab)) | (x >= abc)).astype(np.uint32)
            u = (u << np.uint32(1)) | row
            v = (v << np.uint32(1)) | col
        return u, v

    return _first_distinct_pairs(draw, n_edges, max(2 * n_edges, 1024))


def random_tree(n_nodes: int, seed: int, min_children: int = 1,
                max_children: int = 4) -> np.ndarray:
    """Rooted tree built breadth-first: root 0; each dequeued node gets
    ``U{min..max}`` children, ids in creation order; stops at ``n_nodes``.

    Returns the edges ``(parent, child)``.  Because ids are handed out in
    creation order and the queue is FIFO, node ``j`` is the j-th node to be
    dequeued, so the children of ``j`` are a contiguous id range.
    """
    if n_nodes < 1:
        raise ValueError("need at least one node")
    counts = bounded_u32(stream_u64(subkey(seed, 4), 0, n_nodes),
                         max_children - min_children + 1).astype(np.int64)
    counts += min_children
    parents = np.repeat(np.arange(n_nodes, dtype=np.uint32), counts)[:n_nodes - 1]
    out = np.empty((n_nodes - 1, 2), dtype=np.uint32)
    out[:, 0] = parents
    out[:, 1] = np.arange(1, n_nodes, dtype=np.uint32)
    return out


def zipf_ids(n_ids: int, s: float, key: int, start: int, count: int) -> np.ndarray:
    """Ids ``rank - 1`` with rank drawn from Zipf(s) on ``1..n_ids`` by
    inverse CDF (double table, binary search)."""
    w = np.arange(1, n_ids + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    x = unit_double(stream_u64(key, start, count))
    return np.minimum(np.searchsorted(cdf, x, side="right"), n_ids - 1).astype(np.uint32)


def zipf_pairs(n_ids: int, n_pairs: int, s: float, seed: int, tag: int,
               orient: str = "literal") -> np.ndarray:
    """``n_pairs`` distinct non-self pairs with Zipf(s) endpoints.

    ``orient`` selects how a drawn pair becomes a tuple:
      * ``"literal"``  both endpoints Zipf, kept as drawn;
      * ``"by_rank"``  both endpoints Zipf, ordered low id -> high id
        (the relation is acyclic);
      * ``"src_zipf"`` Zipf source, uniform target.
    """
    ku, kv = subkey(seed, 16 + 2 * tag), subkey(seed, 17 + 2 * tag)

    def draw(start, count):
        u = zipf_ids(n_ids, s, ku, start, count)
        if orient == "src_zipf":
            v = bounded_u32(stream_u64(kv, start, count), n_ids)
        else:
            v = zipf_ids(n_ids, s, kv, start, count)
        if orient == "by_rank":
            u, v = np.minimum(u, v), np.maximum(u, v)
        return u, v

    return _first_distinct_pairs(draw, n_pairs, max(4 * n_pairs, 4096))


def batched_reach_instances(n_inst: int, seed: int, lo: int = 32, hi: int = 4096):
    """Independent Reach inputs: instance k has ``n_k`` nodes, log-uniform in
    ``[lo, hi]``, and ``floor(U(2,4) * n_k)`` distinct non-self uniform edges.

    Returns ``(node_counts, edge_lists)``.
    """
    nodes, edges = [], []
    for k in range(n_inst):
        ks = splitmix64_scalar((seed ^ k) & _MASK64)
        r = unit_double(stream_u64(ks, 0, 2))
        n = int(math.floor(math.exp(math.log(lo) + r[0] * (math.log(hi) - math.log(lo)))))
        n = max(lo, min(hi, n))
        m = int(math.floor((2.0 + 2.0 * r[1]) * n))
        nodes.append(n)
        edges.append(erdos_renyi(n, m, ks))
    return np.asarray(nodes, dtype=np.int64), edges


# ---------------------------------------------------------------------------
# Named workloads.  Each is a plain dict: program name plus EDB arrays.

REACH = "reach"
SG = "sg"


def reach_er_1000():
    """Reach on a directed Erdos-Renyi graph: 1,000 nodes, 3,000 edges."""
    return {"program": REACH, "n_nodes": 1000,
            "edb": {"Edge": erdos_renyi(1000, 3000, 0xC1)}}


def reach_rmat16():
    """Reach on an R-MAT graph (0.57/0.19/0.19/0.05): 2^16 nodes, 200,000 edges."""
    return {"program": REACH, "n_nodes": 1 << 16,
            "edb": {"Edge": rmat(16, 200_000, 0xC2A)}}


def sg_tree_50k():
    """Same-generation on a random breadth-first tree of 50,000 nodes,
    branching 1-4 uniform."""
    return {"program": SG, "n_nodes": 50_000,
            "edb": {"Edge": random_tree(50_000, 0xC2B)}}


def reach_er_2p22():
    """Reach on a subcritical directed ER graph: 2^22 nodes, 0.9 * 2^22 edges."""
    n = 1 << 22
    return {"program": REACH, "n_nodes": n,
            "edb": {"Edge": erdos_renyi(n, int(0.9 * n), 0xC5)}}


def cspa(log2_ids: int = 14, orient: str = "literal", seed: int = 0xC3):
    """The CSPA-shaped points-to program's EDB: Zipf(1.2) endpoints over
    ``2^log2_ids`` variable ids, Assign and Dereference at the density of
    400,000 and 150,000 pairs per 2^20 ids (so 6,250 and 2,343 pairs at
    2^14).  Join candidates grow about sevenfold per doubling of the id
    space (1.7e10 duplicates for 9.2e6 tuples at 2^14, literal reading),
    and at 2^15 one iteration of every reading already needs more than
    200 GB of candidates, so the default is the largest power of two where
    the literal reading stays under 5e10 candidates and 2e9 tuples."""
    ids = 1 << log2_ids
    na, nd = int(400_000 * ids / (1 << 20)), int(150_000 * ids / (1 << 20))
    return {"program": "cspa_shaped", "n_ids": ids, "orient": orient,
            "edb": {"Assign": zipf_pairs(ids, na, 1.2, seed, 0, orient=orient),
                    "Dereference": zipf_pairs(ids, nd, 1.2, seed, 1, orient=orient)}}


def scaled_rmat(scale: int, n_edges: int, seed: int = 0xC2A):
    return {"program": REACH, "n_nodes": 1 << scale,
            "edb": {"Edge": rmat(scale, n_edges, seed)}}


def scaled_tree(n_nodes: int, seed: int = 0xC2B):
    return {"program": SG, "n_nodes": n_nodes,
            "edb": {"Edge": random_tree(n_nodes, seed)}}
