"""Fused small iterations (HL_FLAG_FUSED, HL_FLAG_HIP_GRAPH) against the
oracle, bit-exact: final IDB sets and per-iteration delta sizes, on inputs
whose long tails of small deltas take the fused launch.  Covers 32- and
64-bit keys, hash and learned probes, HIP graph capture and replay, a
two-join rule with a filter (same-generation), a one-atom recursive rule,
two IDB relations, batched instances, and an iteration whose candidates
overflow the LDS capacity and is rerun on the multi-kernel path."""

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


def check_same(program, edb, idb, **kw):
    import torch
    import paper_2311_02206_amd as pkg
    torch.cuda.set_device(0)
    want = oracle.evaluate(program, edb, idb, max_iterations=100_000)
    rels, deltas, st = pkg.evaluate(program, edb, idb, device=0,
                                    stream=torch.cuda.current_stream(), **kw)
    for name in idb:
        assert np.array_equal(rels[name], want.relations[name]), name
        assert deltas[name] == want.deltas[name], name
    assert st.iterations == want.iterations
    return st


MODES = {
    "fused": dict(fused=True),
    "graph": dict(fused=True, hip_graph=True),
    "graph_learned": dict(fused=True, hip_graph=True, learned=True),
}


def subcritical_er(n, seed, spread=1):
    """Erdos-Renyi graph with 0.9 n edges: a closure with a long tail of
    small deltas.  spread > 1 relabels ids i -> spread * i + 7, which widens
    the packed keys without changing the graph."""
    e = workloads.erdos_renyi(n, int(0.9 * n), seed).astype(np.uint64)
    return (e * spread + (7 if spread > 1 else 0)).astype(np.uint32)


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("spread", [1, 40])
def test_reach_long_tail(mode, spread):
    say(f"fused reach, subcritical ER 2^14, spread {spread}, {mode}")
    E = subcritical_er(1 << 14, 0xC5, spread)
    st = check_same(PROG["reach"], {"Edge": E}, {"Reach": 2}, **MODES[mode])
    assert st.key_bytes == (4 if spread == 1 else 8)
    assert st.fused_iterations > 10
    if "graph" in mode:
        # the graph of each buffer parity is captured once and then replayed
        assert 1 <= st.graph_captures < st.fused_iterations


def test_fused_off_gives_the_same_counts():
    """The fused and multi-kernel paths agree on every statistic that
    describes the result: iterations, new tuples and join outputs."""
    import torch
    import paper_2311_02206_amd as pkg
    say("fused vs plain statistics")
    E = subcritical_er(1 << 14, 0xC6)
    out = {}
    for k, kw in (("plain", {}), ("fused", dict(fused=True))):
        out[k] = pkg.evaluate(PROG["reach"], {"Edge": E}, {"Reach": 2}, device=0,
                              stream=torch.cuda.current_stream(), **kw)
    (r0, d0, s0), (r1, d1, s1) = out["plain"], out["fused"]
    assert np.array_equal(r0["Reach"], r1["Reach"]) and d0 == d1
    assert s0.iterations == s1.iterations and s0.idb_tuples == s1.idb_tuples
    assert s0.join_outputs == s1.join_outputs and s0.candidates == s1.candidates
    assert s0.fused_iterations == 0 and s1.fused_iterations > 10


def overflow_graph():
    """A path of 300 nodes (small deltas for 300 iterations) beside a hub
    whose rate of join outputs jumps: 64 leaves point at Y, Y starts a chain
    of 5 nodes that fans out to 64 nodes.  When Y first reaches the fan, 64
    delta tuples produce 64 * 64 outputs, more than a 1,024-key fused
    launch holds, while the previous iteration predicted about a hundred."""
    path = [(i, i + 1) for i in range(300)]
    base = 1000
    y = base
    leaves = [(base + 1 + i, y) for i in range(64)]
    chain = [(y + 100 + i, y + 101 + i) for i in range(5)]
    chain = [(y, y + 100)] + chain
    fan = [(y + 105, y + 200 + i) for i in range(64)]
    return np.array(path + leaves + chain + fan, dtype=np.uint32)


@pytest.mark.parametrize("graph", [False, True])
def test_overflow_reruns_the_iteration(graph):
    say(f"fused overflow fallback, graph={graph}")
    E = overflow_graph()
    st = check_same(PROG["reach"], {"Edge": E}, {"Reach": 2}, fused=True, hip_graph=graph,
                    fused_capacity=1024)
    assert st.fused_overflows >= 1
    assert st.fused_iterations > 100


@pytest.mark.parametrize("mode", ["fused", "graph"])
def test_sg_two_joins_with_filter(mode):
    say(f"fused sg tree 300, {mode}")
    wl = workloads.scaled_tree(300, seed=17)
    st = check_same(PROG["sg"], wl["edb"], {"SG": 2}, **MODES[mode])
    total, cf = oracle.sg_tree_closed_form(wl["edb"]["Edge"])
    assert st.idb_tuples == total
    assert st.fused_iterations > 0


def test_sg_deep_narrow_tree():
    """A tree of long chains: same-generation deltas stay small for many
    iterations, all of them fused."""
    say("fused sg, chains")
    edges = []
    nxt = 1
    for c in range(6):  # six chains of 120 nodes under the root
        prev = 0
        for d in range(120):
            edges.append((prev, nxt))
            prev = nxt
            nxt += 1
    E = np.array(edges, dtype=np.uint32)
    st = check_same(PROG["sg"], {"Edge": E}, {"SG": 2}, fused=True, hip_graph=True)
    assert st.fused_iterations > 100


def test_one_atom_recursive_rule():
    """T(x, y) :- T(y, x) is a projection of the delta with no join."""
    say("fused symmetric closure")
    prog = "T(x, y) :- E(x, y).\nT(x, y) :- T(y, x).\nT(x, z) :- T(x, y), E(y, z).\n"
    E = subcritical_er(3000, 0xC7)
    st = check_same(prog, {"E": E}, {"T": 2}, fused=True, hip_graph=True)
    assert st.fused_iterations > 0


def test_two_idb_relations():
    """Odd and even path lengths: each iteration grows one relation from
    the other's delta, so the buffers of the two relations swap on
    alternate iterations."""
    say("fused odd/even paths")
    prog = ("Odd(x, y) :- E(x, y).\nEven(x, y) :- Odd(x, z), E(z, y).\n"
            "Odd(x, y) :- Even(x, z), E(z, y).\n")
    E = subcritical_er(4000, 0xC8)
    st = check_same(prog, {"E": E}, {"Odd": 2, "Even": 2}, fused=True, hip_graph=True)
    assert st.fused_iterations > 0


def test_empty_and_tiny_inputs():
    say("fused edge cases")
    for E in (np.array([[5, 5]], dtype=np.uint32), np.array([[0, 1]], dtype=np.uint32),
              np.array([[0, 1], [1, 0]], dtype=np.uint32),
              np.array([[i, i + 1] for i in range(40)], dtype=np.uint32)):
        check_same(PROG["reach"], {"Edge": E}, {"Reach": 2}, fused=True, hip_graph=True)


def test_tail_folds_into_full_mid_run():
    """A directed path of 800 nodes: 800 fused iterations whose deltas sum
    to 319,600 tuples, more than one tail run holds (2^18 keys), so the tail
    is folded into full while the fused iterations go on."""
    say("fused path 800, tail fold")
    E = np.array([[i, i + 1] for i in range(799)], dtype=np.uint32)
    st = check_same(PROG["reach"], {"Edge": E}, {"Reach": 2}, fused=True, hip_graph=True)
    assert st.idb_tuples == 800 * 799 // 2
    assert st.fused_iterations > 700
