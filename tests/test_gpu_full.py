"""GPU parity at the benchmark's full sizes, in the launch configuration
bench.py times.  The std::set oracle cannot run at these sizes (tens of GB
and hours), so the references are exact independent computations that the
oracle's pins tie to it, and every row of every output is compared:
  * Reach: for every source, a breadth-first search over the edges marks
    the reachable nodes, and that source's fetched rows must be exactly the
    marked nodes (oracle.reach_verify: strictly increasing, all marked, as
    many as marked); the shortest-distance histogram gives every
    per-iteration delta size;
  * SG on a tree: every fetched row must be a pair of distinct nodes of equal
    depth (oracle.sg_tree_verify), the rows strictly increasing, and their
    number the closed form's, which together is set equality; the closed
    form also gives every per-iteration delta;
  * the CSPA-shaped program: naive evaluation over boolean matrices of the
    active ids (every tuple and every per-iteration delta);
  * the 4,096-instance batch: every instance's rows against its own
    reachability searches, and the batch's per-iteration deltas against
    the sum of the instances' distance histograms, in both engine forms
    bench.py times.
"""

import os
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROG = {n: open(os.path.join(ROOT, "workloads", "programs", n + ".dl")).read()
        for n in ("reach", "sg", "cspa_shaped")}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def engine(program, edb, idb, learned=False, **kw):
    import torch
    import paper_2311_02206_amd as pkg
    torch.cuda.set_device(0)
    e = pkg.Engine(device=0, stream=torch.cuda.current_stream(), learned=learned, **kw)
    for n in edb:
        e.declare(n, 2, True)
    for n, a in idb.items():
        e.declare(n, a, False)
    for n, rows in edb.items():
        e.load(n, rows)
    e.program(program)
    return e


def verify_all_rows(n_nodes, E, R, deltas, doubling=False):
    """Every row of a fetched Reach relation against per-source searches,
    and the per-iteration delta sizes against the distance histogram."""
    bad, first, hist = oracle.reach_verify(n_nodes, E, R)
    assert bad == 0, f"{bad} sources differ, first {first}"
    assert len(R) == sum(hist)
    want = (oracle.doubling_deltas_from_histogram(hist) if doubling
            else oracle.reach_deltas_from_histogram(hist))
    assert deltas == want


def check_reach(wl, learned=False, **kw):
    E = wl["edb"]["Edge"]
    e = engine(PROG["reach"], wl["edb"], {"Reach": 2}, learned=learned, **kw)
    try:
        st = e.run()
        say(f"  ran: {st.idb_tuples} tuples, {st.iterations} iterations, {st.seconds:.3f} s")
        R = e.fetch("Reach")
        assert e.count("Reach") == len(R)
        verify_all_rows(wl["n_nodes"], E, R, e.iteration_counts("Reach", 0))
        say(f"  all {len(R)} rows verified")
        return st
    finally:
        e.close()


def test_reach_rmat16_200k():
    say("reach rmat 2^16 / 200k")
    wl = workloads.reach_rmat16()
    st = check_reach(wl)
    assert st.key_bytes == 4


def test_sg_tree_50k():
    say("sg tree 50k")
    wl = workloads.sg_tree_50k()
    E = wl["edb"]["Edge"]
    e = engine(PROG["sg"], wl["edb"], {"SG": 2})
    try:
        st = e.run()
        say(f"  ran: {st.idb_tuples} tuples, {st.iterations} iterations, {st.seconds:.3f} s")
        total, deltas = oracle.sg_tree_closed_form(E)
        assert e.count("SG") == total
        assert e.iteration_counts("SG", 0) == deltas
        S = e.fetch("SG")
        assert len(S) == total
        # every row a pair of distinct same-depth nodes, strictly increasing:
        # with the closed-form count, the fetched set is the definition's
        bad, first = oracle.sg_tree_verify(E, S)
        assert bad == 0, f"{bad} rows fail the same-generation predicate, first {first}"
        say(f"  all {len(S)} rows verified")
        n = int(E.max()) + 1
        depth = np.zeros(n, dtype=np.int64)
        for p, c in E.tolist():
            depth[c] = depth[p] + 1
        # every row of a few nodes, spelled out: the other nodes of its depth
        for v in (1, 7, 1234, 49_999):
            lo, hi = np.searchsorted(S[:, 0], [v, v + 1])
            want = np.nonzero((depth == depth[v]) & (np.arange(n) != v))[0]
            assert np.array_equal(S[lo:hi, 1].astype(np.int64), want)
    finally:
        e.close()


ER_MODES = {
    "plain": {},
    "learned": {"learned": True},
    # every option on: learned index, fused small iterations from HIP graphs
    "all_on": {"learned": True, "fused": True, "hip_graph": True},
    # new tuples sorted in 2^20-key chunks: chunked iterations fold the
    # tail run into full before their membership tests
    "chunked": {"sort_chunk_log2": 20},
}


@pytest.mark.parametrize("mode", list(ER_MODES))
def test_reach_er_2p22_subcritical(mode):
    say(f"reach er 2^22 subcritical, {mode}")
    wl = workloads.reach_er_2p22()
    kw = dict(ER_MODES[mode])
    st = check_reach(wl, **kw)
    assert st.key_bytes == 8
    if mode == "all_on":
        assert st.fused_iterations > 30 and st.graph_captures >= 1


NONLINEAR = "T(x, y) :- E(x, y).\nT(x, y) :- T(x, z), T(z, y)."


@pytest.mark.parametrize("learned", [False, True])
def test_nonlinear_closure_er_2p22(learned):
    """The nonlinear closure on the 2^22-node ER graph, where the growing
    relation is itself the join's inner (hash rebuilt, or model refitted,
    after every merge): every row against per-source searches, and the
    per-iteration deltas from the distance histogram (doubling)."""
    say(f"nonlinear closure er 2^22, learned={learned}")
    wl = workloads.reach_er_2p22()
    E = wl["edb"]["Edge"]
    e = engine(NONLINEAR, {"E": E}, {"T": 2}, learned=learned)
    try:
        st = e.run()
        say(f"  ran: {st.idb_tuples} tuples, {st.iterations} iterations, {st.seconds:.3f} s")
        T = e.fetch("T")
        assert e.count("T") == len(T)
        verify_all_rows(wl["n_nodes"], E, T, e.iteration_counts("T", 0), doubling=True)
        say(f"  all {len(T)} rows verified")
    finally:
        e.close()


_CSPA_WANT = {}


@pytest.mark.parametrize("learned", [False, True])
def test_cspa_literal_2p14(learned):
    """The CSPA-shaped program at the size bench.py times (2^14 ids, literal
    Zipf reading, 6,250 Assign and 2,343 Dereference pairs: 9.2e6 tuples from
    1.7e10 join candidates).  The std::set oracle would take hours; the
    reference is the oracle's naive evaluator over boolean matrices, pinned
    to the std::set oracle and brute force on smaller inputs."""
    from oracle import matrix_naive
    say(f"cspa literal 2^14, learned={learned}")
    wl = workloads.cspa(14)
    idb = {"ValueFlow": 2, "ValueAlias": 2, "MemoryAlias": 2}
    if not _CSPA_WANT:
        _CSPA_WANT["r"] = matrix_naive.evaluate(PROG["cspa_shaped"], wl["edb"], idb)
    want = _CSPA_WANT["r"]
    e = engine(PROG["cspa_shaped"], wl["edb"], idb, learned=learned)
    try:
        st = e.run()
        say(f"  ran: {st.idb_tuples} tuples, {st.iterations} iterations, {st.seconds:.3f} s, "
            f"{st.candidates} candidates")
        assert st.iterations == want.iterations
        for n in idb:
            assert e.iteration_counts(n, 0) == want.deltas[n], n
            assert np.array_equal(e.fetch(n), want.relations[n]), n
    finally:
        e.close()


def verify_batch(e, nodes, edges, group_rows=200_000_000):
    """Every instance's rows against its own reachability searches (fetched
    and checked in groups of instances to bound host memory), and the
    batch's per-iteration deltas against the summed distance histograms."""
    k, total, hist = 0, 0, np.zeros(1 << 12, dtype=np.int64)
    while k < len(nodes):
        group, rows, n_rows = [], [], 0
        while k < len(nodes) and (not group or n_rows < group_rows):
            r = e.fetch_batched("Reach", k)
            group.append(k)
            rows.append(r)
            n_rows += len(r)
            k += 1
        bad, first, h = oracle.reach_verify_many(nodes[group], [edges[q] for q in group], rows)
        assert bad == 0, f"{bad} instances differ, first {group[first] if first >= 0 else first}"
        hist[:len(h)] += h
        total += n_rows
    assert total == e.count("Reach")
    last = int(np.nonzero(hist)[0].max())
    assert e.iteration_counts("Reach", 0) == oracle.reach_deltas_from_histogram(hist[:last + 1])
    return total


@pytest.mark.parametrize("form", ["plain", "fused_graph"])
def test_batched_reach_4096_instances(form):
    """4,096 independent Reach instances (log-uniform 32..4096 nodes, 2-4x
    edges) in one batched fixpoint, in both forms bench.py times (EBM growth
    1.5; fused small iterations from HIP graphs or not): every row of every
    instance."""
    import torch
    import paper_2311_02206_amd as pkg
    say(f"batched reach, 4096 instances, {form}")
    nodes, edges = workloads.batched_reach_instances(4096, seed=0xC4)
    nodes = np.asarray(nodes)
    kw = {"fused": True, "hip_graph": True} if form == "fused_graph" else {}
    e = pkg.Engine(device=0, stream=torch.cuda.current_stream(), ebm_k=1.5, **kw)
    try:
        e.declare("Edge", 2, True)
        e.declare("Reach", 2, False)
        e.batch_layout(nodes)
        e.load_batched("Edge", edges)
        e.program(PROG["reach"])
        st = e.run()
        say(f"  ran: {st.idb_tuples} tuples, {st.iterations} iterations, {st.seconds:.3f} s, "
            f"{st.fused_iterations} fused")
        if form == "fused_graph":
            assert st.fused_iterations > 0
        n = verify_batch(e, nodes, edges)
        say(f"  all {n} rows of 4096 instances verified")
    finally:
        e.close()


def test_cspa_literal_2p15_chunked_joins():
    """CSPA at 2^15 ids (1.2e11 join outputs: no single join's output fits
    the device, so every large join runs in chunks).  Reference: the
    oracle's matrix evaluator, stored by tests/golden/make_cspa_2p15.py as
    sizes, per-iteration deltas and a SHA-256 of each relation's sorted rows
    (compared here with the fetched rows, so every row is checked)."""
    import hashlib
    import json
    say("cspa literal 2^15, chunked joins")
    want = json.load(open(os.path.join(ROOT, "tests", "golden", "cspa_2p15.json")))
    wl = workloads.cspa(15)
    idb = {"ValueFlow": 2, "ValueAlias": 2, "MemoryAlias": 2}
    e = engine(PROG["cspa_shaped"], wl["edb"], idb)
    try:
        st = e.run()
        say(f"  ran: {st.idb_tuples} tuples, {st.iterations} iterations, {st.seconds:.3f} s, "
            f"{st.join_outputs} join outputs, peak {st.peak_bytes / 1e9:.1f} GB")
        assert st.iterations == want["iterations"]
        for n in idb:
            w = want["relations"][n]
            assert e.count(n) == w["size"], n
            assert e.iteration_counts(n, 0) == w["deltas"], n
            rows = np.ascontiguousarray(e.fetch(n), dtype=np.uint32)
            assert hashlib.sha256(rows.tobytes()).hexdigest() == w["sha256"], n
    finally:
        e.close()
