"""Pins of the whole-relation checkers (oracle/closure_check.cpp) that the
full-size GPU tests use: on small inputs they must accept exactly the
std::set oracle's result (an independent algorithm), return its distance
histogram, and reject every planted mistake (a missing row, an extra row, a
wrong target, a duplicate, a row out of order, a wrong instance)."""

import os

import numpy as np
import pytest

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROG = {n: open(os.path.join(ROOT, "workloads", "programs", n + ".dl")).read()
        for n in ("reach", "sg")}


def closure(n, E):
    return oracle.evaluate(PROG["reach"], {"Edge": E}, {"Reach": 2}).relations["Reach"]


def graphs():
    yield "er", 300, workloads.erdos_renyi(300, 700, 3)
    yield "rmat", 1 << 9, workloads.scaled_rmat(9, 1500, seed=4)["edb"]["Edge"]
    cyc = np.array([[i, (i + 1) % 40] for i in range(40)], np.uint32)
    yield "cycle", 50, cyc
    yield "empty", 10, np.zeros((0, 2), np.uint32)
    yield "loop", 5, np.array([[2, 2]], np.uint32)


@pytest.mark.parametrize("name,n,E", list(graphs()), ids=[g[0] for g in graphs()])
def test_reach_verify_accepts_oracle(name, n, E):
    R = closure(n, E)
    bad, first, hist = oracle.reach_verify(n, E, R, threads=4)
    assert (bad, first) == (0, -1)
    total, want_hist = oracle.reach_bfs_histogram(n, E, threads=2)
    assert hist == want_hist and sum(hist) == total == len(R)


def sorted_insert(R, row):
    key = (R[:, 0].astype(np.uint64) << np.uint64(32)) | R[:, 1]
    k = (np.uint64(row[0]) << np.uint64(32)) | np.uint64(row[1])
    p = int(np.searchsorted(key, k))
    return np.insert(R, p, np.array(row, np.uint32), axis=0)


def test_reach_verify_rejects_planted_mistakes():
    n = 300
    E = workloads.erdos_renyi(300, 700, 3)
    R = closure(n, E)
    assert len(R) > 1000
    rng = np.random.default_rng(0)
    # a dropped row: exactly its source mismatches
    i = int(rng.integers(len(R)))
    bad, first, _ = oracle.reach_verify(n, E, np.delete(R, i, axis=0), threads=3)
    assert (bad, first) == (1, int(R[i, 0]))
    # an extra pair that is not reachable (inserted in sorted position)
    reach = {tuple(r) for r in R.tolist()}
    extra = next((s, t) for s in range(n) for t in range(n) if (s, t) not in reach)
    bad, first, _ = oracle.reach_verify(n, E, sorted_insert(R, extra), threads=3)
    assert (bad, first) == (1, extra[0])
    # a target replaced by an unreachable node (order kept, count kept)
    for s in range(n):
        rows = R[R[:, 0] == s, 1]
        if 0 < len(rows) < n - 1:
            gaps = sorted(set(range(n)) - set(rows.tolist()))
            j = int(np.searchsorted(R[:, 0], s)) + len(rows) - 1
            if gaps[-1] > rows[-1]:
                W = R.copy()
                W[j, 1] = gaps[-1]
                bad, first, _ = oracle.reach_verify(n, E, W, threads=3)
                assert (bad, first) == (1, s)
                break
    else:
        pytest.fail("no source to plant a wrong target in")
    # a duplicate row, and two rows out of order: not a sorted set
    with pytest.raises(ValueError):
        oracle.reach_verify(n, E, np.insert(R, 5, R[5], axis=0))
    W = R.copy()
    W[[10, 11]] = W[[11, 10]]
    with pytest.raises(ValueError):
        oracle.reach_verify(n, E, W)
    # an id outside the graph
    W = np.concatenate([R, np.array([[n - 1, n]], np.uint32)])
    with pytest.raises(ValueError):
        oracle.reach_verify(n, E, W)


def test_reach_verify_many():
    nodes, edges = workloads.batched_reach_instances(12, seed=11, lo=8, hi=120)
    rows = [closure(int(n), e) for n, e in zip(nodes, edges)]
    bad, first, hist = oracle.reach_verify_many(nodes, edges, rows, threads=4)
    assert (bad, first) == (0, -1)
    want = np.zeros(len(hist) + 64, dtype=np.int64)
    for n, e in zip(nodes, edges):
        _, h = oracle.reach_bfs_histogram(int(n), e, threads=1)
        want[:len(h)] += h
    assert hist == want[:len(hist)].tolist()
    # instance 7 loses a row, instance 3 gains one: both are found
    rows[7] = rows[7][1:]
    present = {tuple(r) for r in rows[3].tolist()}
    extra = next((s, t) for s in range(int(nodes[3])) for t in range(int(nodes[3]))
                 if (s, t) not in present)
    rows[3] = sorted_insert(rows[3], extra)
    bad, first, _ = oracle.reach_verify_many(nodes, edges, rows, threads=4)
    assert (bad, first) == (2, 3)


@pytest.mark.parametrize("n", [2, 17, 400, 1500])
def test_sg_tree_verify(n):
    t = workloads.random_tree(n, seed=n)
    S = oracle.evaluate(PROG["sg"], {"Edge": t}, {"SG": 2}).relations["SG"]
    assert oracle.sg_tree_verify(t, S, threads=3) == (0, -1)
    total, _ = oracle.sg_tree_closed_form(t)
    assert total == len(S)
    if len(S) < 4:
        return
    # a pair across depths, the reflexive pair, and a root pair are rejected;
    # a missing row keeps the predicate but fails the closed-form count
    depth = np.zeros(n, np.int64)
    for p, c in t.tolist():
        depth[c] = depth[p] + 1
    W = S.copy()
    x, y = int(W[-1, 0]), int(W[-1, 1])
    other = [v for v in range(n) if depth[v] != depth[x] and v > y]
    if other:
        W[-1, 1] = other[0]
        assert oracle.sg_tree_verify(t, W)[0] == 1
    W = sorted_insert(S, (x, x)) if (x, x) not in {tuple(r) for r in S.tolist()} else S
    assert oracle.sg_tree_verify(t, W)[0] == 1
    W = sorted_insert(S, (0, 1)) if depth[1] == 0 else sorted_insert(S, (0, n - 1))
    assert oracle.sg_tree_verify(t, W)[0] >= 1
    assert oracle.sg_tree_verify(t, S[1:])[0] == 0 and len(S[1:]) != total
    with pytest.raises(ValueError):
        oracle.sg_tree_verify(t, S[::-1])


@pytest.mark.parametrize("n", [0, 1, 2, 7, 4097, 1_000_003])
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_host_sort_and_merge(n, threads):
    """The host side of the sort/merge microbenchmark equals numpy's sort
    and a sorted concatenation (odd run counts, ties, extremes)."""
    rng = np.random.default_rng(n * 10 + threads)
    a = rng.integers(0, 2**64 - 1, size=n, dtype=np.uint64, endpoint=True)
    if n > 4:
        a[:3] = [0, 2**64 - 1, 5]
        a[3:5] = 5
    want = np.sort(a)
    oracle.host_sort_u64(a, threads)
    assert np.array_equal(a, want)
    x = np.sort(rng.integers(0, 50, size=n // 3, dtype=np.uint64))
    y = np.sort(rng.integers(0, 50, size=n - n // 3, dtype=np.uint64))
    out = np.empty(n, dtype=np.uint64)
    oracle.host_merge_u64(x, y, out, threads)
    assert np.array_equal(out, np.sort(np.concatenate([x, y])))
    assert oracle.host_alloc_init(max(n, 1) * 8, threads) >= 0
