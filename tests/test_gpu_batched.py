"""Batched evaluation of many independent instances in one fixpoint: each
instance's part of the result must equal that instance evaluated alone by the
oracle (bit-exact), for Reach and SG."""

import os
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROG = {n: open(os.path.join(ROOT, "workloads", "programs", n + ".dl")).read()
        for n in ("reach", "sg")}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def batched_engine(program, instances, ranges, idb, learned=False, **kw):
    import torch
    import paper_2311_02206_amd as pkg
    torch.cuda.set_device(0)
    e = pkg.Engine(device=0, stream=torch.cuda.current_stream(), learned=learned, **kw)
    e.declare("Edge", 2, True)
    for n in idb:
        e.declare(n, 2, False)
    e.batch_layout(ranges)
    e.load_batched("Edge", instances)
    e.program(program)
    return e


_SMALL = {}


def small_batch():
    """64 instances of 32..600 nodes (the std::set oracle stays in seconds),
    with the oracle's result of each, computed once."""
    if not _SMALL:
        nodes, edges = workloads.batched_reach_instances(64, seed=0xC4, lo=32, hi=600)
        want = [oracle.evaluate(PROG["reach"], {"Edge": ed}, {"Reach": 2}).relations["Reach"]
                for ed in edges]
        _SMALL.update(nodes=nodes, edges=edges, want=want)
    return _SMALL["nodes"], _SMALL["edges"], _SMALL["want"]


@pytest.mark.parametrize("mode", ["plain", "learned", "fused_graph"])
def test_batched_reach_matches_per_instance_oracle(mode):
    say(f"batched reach, 64 instances, {mode}")
    nodes, edges, want = small_batch()
    kw = {"fused": True, "hip_graph": True} if mode == "fused_graph" else {}
    e = batched_engine(PROG["reach"], edges, nodes, {"Reach": 2}, mode == "learned", **kw)
    try:
        st = e.run()
        if mode == "fused_graph":
            assert st.fused_iterations > 0
        total = 0
        for k in range(len(edges)):
            got = e.fetch_batched("Reach", k)
            assert np.array_equal(got, want[k]), k
            total += len(got)
        assert e.count("Reach") == total == st.idb_tuples
    finally:
        e.close()


def test_batched_reach_iteration_totals():
    """Per-iteration totals of the batch = sums of the instances' own
    per-iteration deltas (BFS distance histograms), padded with zeros."""
    say("batched reach iteration totals, 200 instances")
    nodes, edges = workloads.batched_reach_instances(200, seed=7)
    e = batched_engine(PROG["reach"], edges, nodes, {"Reach": 2})
    try:
        e.run()
        got = e.iteration_counts("Reach", 0)
        want = np.zeros(len(got), dtype=np.int64)
        for k in range(len(edges)):
            _, hist = oracle.reach_bfs_histogram(int(nodes[k]), edges[k], threads=4)
            d = oracle.reach_deltas_from_histogram(hist)
            assert len(d) <= len(got)
            want[:len(d)] += d
        assert got == want.tolist()
    finally:
        e.close()


def test_batched_sg_trees():
    say("batched sg on 30 trees")
    trees = [workloads.random_tree(int(n), seed=int(n)) for n in np.linspace(2, 3000, 30)]
    ranges = [len(t) + 1 for t in trees]
    e = batched_engine(PROG["sg"], trees, ranges, {"SG": 2})
    try:
        e.run()
        for k, t in enumerate(trees):
            total, _ = oracle.sg_tree_closed_form(t) if len(t) else (0, [0])
            got = e.fetch_batched("SG", k)
            assert len(got) == total
            if ranges[k] <= 600:
                want = oracle.evaluate(PROG["sg"], {"Edge": t}, {"SG": 2})
                assert np.array_equal(got, want.relations["SG"])
    finally:
        e.close()


def test_batch_errors():
    import torch
    import paper_2311_02206_amd as pkg
    say("batch errors")
    with pkg.Engine(device=0, stream=torch.cuda.current_stream()) as e:
        e.declare("Edge", 2, True)
        e.declare("Reach", 2, False)
        with pytest.raises(pkg.HlError):
            e.load_batched("Edge", [np.array([[0, 1]], np.uint32)])  # no layout yet
        e.batch_layout([4, 4])
        with pytest.raises(pkg.HlError) as ei:
            e.load_batched("Edge", [np.array([[0, 5]], np.uint32), np.zeros((0, 2), np.uint32)])
        assert ei.value.code == pkg.hisalog.HL_E_INVALID  # id 5 outside range 4
        e.load_batched("Edge", [np.array([[0, 1], [1, 2]], np.uint32),
                                np.array([[3, 0]], np.uint32)])
        e.program(PROG["reach"])
        e.run()
        assert e.fetch_batched("Reach", 0).tolist() == [[0, 1], [0, 2], [1, 2]]
        assert e.fetch_batched("Reach", 1).tolist() == [[3, 0]]
        with pytest.raises(pkg.HlError):
            e.fetch_batched("Reach", 2)


def test_batched_empty_and_tiny_instances():
    """Instances with no edges, a single node, a self-loop only, and a
    cycle, side by side: each instance's result is its own closure, and
    instances never mix (the closure of the union is the union of the
    closures when no id is shared)."""
    import torch
    import paper_2311_02206_amd as pkg
    say("batched: empty and tiny instances")
    ranges = [5, 1, 3, 4, 1]
    edges = [np.zeros((0, 2), np.uint32),                     # no edges
             np.zeros((0, 2), np.uint32),                     # one node, no edges
             np.array([[2, 2]], np.uint32),                   # a self-loop only
             np.array([[0, 1], [1, 2], [2, 3], [3, 0]], np.uint32),  # a 4-cycle
             np.array([[0, 0]], np.uint32)]                   # one node with a loop
    with pkg.Engine(device=0, stream=torch.cuda.current_stream()) as e:
        e.declare("Edge", 2, True)
        e.declare("Reach", 2, False)
        e.batch_layout(ranges)
        e.load_batched("Edge", edges)
        e.program(PROG["reach"])
        for _ in range(2):
            e.run()
            for k, ed in enumerate(edges):
                want = oracle.evaluate(PROG["reach"], {"Edge": ed}, {"Reach": 2}).relations["Reach"]
                got = e.fetch_batched("Reach", k)
                assert np.array_equal(got, want), k
                assert e.batch_count("Reach", k) == len(want)
        assert e.count("Reach") == 1 + 16 + 1


@pytest.mark.parametrize("mode", ["plain", "fused_graph"])
def test_batched_unary_edb(mode):
    """A unary EDB relation loaded per instance (one or two sources each):
    single-source reachability of every instance against the oracle run on
    that instance alone.  The batched load must read rows of the declared
    arity (one id per row here), not pairs."""
    import torch
    import paper_2311_02206_amd as pkg
    say(f"batched unary EDB, {mode}")
    prog = "R(x) :- S(x).\nR(y) :- R(x), E(x, y).\n"
    nodes, edges = workloads.batched_reach_instances(24, seed=0x51, lo=32, hi=400)
    rng = np.random.default_rng(3)
    srcs = [rng.choice(int(n), size=1 + (k % 2), replace=False).astype(np.uint32).reshape(-1, 1)
            for k, n in enumerate(nodes)]
    kw = {"fused": True, "hip_graph": True} if mode == "fused_graph" else {}
    with pkg.Engine(device=0, stream=torch.cuda.current_stream(), **kw) as e:
        e.declare("E", 2, True)
        e.declare("S", 1, True)
        e.declare("R", 1, False)
        e.batch_layout(nodes)
        e.load_batched("E", edges)
        e.load_batched("S", srcs)
        e.program(prog)
        e.run()
        total = 0
        for k in range(len(nodes)):
            want = oracle.evaluate(prog, {"E": edges[k], "S": srcs[k]}, {"R": 1}).relations["R"]
            got = e.fetch_batched("R", k)
            assert got.shape[1] == 1
            assert np.array_equal(got, want), k
            total += len(want)
        assert e.count("R") == total
