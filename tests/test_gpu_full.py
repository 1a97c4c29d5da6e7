"""GPU parity at the benchmark's full sizes, in the launch configuration
bench.py times (one engine per program, default options).  The std::set
oracle cannot run at these sizes (tens of GB and hours), so the references
are exact independent computations the oracle's pins already tie to it:
  * Reach: per-source BFS gives the tuple count and, through the shortest
    distance histogram, every per-iteration delta size; sampled sources are
    compared row by row;
  * SG on a tree: the closed form gives the count and per-iteration deltas;
    sampled rows are checked against the same-depth definition, and the
    output must be sorted, unique, irreflexive and symmetric;
  * the CSPA-shaped program: naive evaluation over boolean matrices of the
    active ids (every tuple and every per-iteration delta).
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


def check_reach(wl, sources, learned=False, **kw):
    E = wl["edb"]["Edge"]
    e = engine(PROG["reach"], wl["edb"], {"Reach": 2}, learned=learned, **kw)
    try:
        st = e.run()
        say(f"  ran: {st.idb_tuples} tuples, {st.iterations} iterations, {st.seconds:.3f} s")
        total, hist = oracle.reach_bfs_histogram(wl["n_nodes"], E)
        assert e.count("Reach") == total
        assert e.iteration_counts("Reach", 0) == oracle.reach_deltas_from_histogram(hist)
        R = e.fetch("Reach")
        key = (R[:, 0].astype(np.uint64) << np.uint64(32)) | R[:, 1]
        assert np.all(key[1:] > key[:-1])
        for s in sources:
            lo, hi = np.searchsorted(R[:, 0], [s, s + 1])
            assert np.array_equal(R[lo:hi, 1], oracle.reach_from(wl["n_nodes"], E, s)), s
        return st
    finally:
        e.close()


def test_reach_rmat16_200k():
    say("reach rmat 2^16 / 200k")
    wl = workloads.reach_rmat16()
    st = check_reach(wl, [0, 1, 2, 3, 7, 100, 4095, 20000, 65535])
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
        n = int(E.max()) + 1
        depth = np.zeros(n, dtype=np.int64)
        for p, c in E.tolist():
            depth[c] = depth[p] + 1
        key = (S[:, 0].astype(np.uint64) << np.uint64(32)) | S[:, 1]
        assert np.all(key[1:] > key[:-1])
        assert np.all(S[:, 0] != S[:, 1])
        rng = np.random.default_rng(1)
        idx = rng.integers(0, len(S), 100_000)
        assert np.all(depth[S[idx, 0]] == depth[S[idx, 1]])
        # symmetry on the sample
        sw = (S[idx, 1].astype(np.uint64) << np.uint64(32)) | S[idx, 0]
        pos = np.searchsorted(key, sw)
        assert np.all(key[np.minimum(pos, len(key) - 1)] == sw)
        # every row of a sampled node: exactly the other nodes of its depth
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
    st = check_reach(wl, [0, 1, 12345, (1 << 22) - 1], **kw)
    assert st.key_bytes == 8
    if mode == "all_on":
        assert st.fused_iterations > 30 and st.graph_captures >= 1


NONLINEAR = "T(x, y) :- E(x, y).\nT(x, y) :- T(x, z), T(z, y)."


@pytest.mark.parametrize("learned", [False, True])
def test_nonlinear_closure_er_2p22(learned):
    """The nonlinear closure on the 2^22-node ER graph, where the growing
    relation is itself the join's inner (hash rebuilt, or model refitted,
    after every merge): count and per-iteration deltas from the distance
    histogram (doubling), sampled sources row by row."""
    say(f"nonlinear closure er 2^22, learned={learned}")
    wl = workloads.reach_er_2p22()
    E = wl["edb"]["Edge"]
    e = engine(NONLINEAR, {"E": E}, {"T": 2}, learned=learned)
    try:
        st = e.run()
        say(f"  ran: {st.idb_tuples} tuples, {st.iterations} iterations, {st.seconds:.3f} s")
        total, hist = oracle.reach_bfs_histogram(wl["n_nodes"], E)
        assert e.count("T") == total
        assert e.iteration_counts("T", 0) == oracle.doubling_deltas_from_histogram(hist)
        T = e.fetch("T")
        for s in (0, 1, 12345, (1 << 22) - 1):
            lo, hi = np.searchsorted(T[:, 0], [s, s + 1])
            assert np.array_equal(T[lo:hi, 1], oracle.reach_from(wl["n_nodes"], E, s)), s
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


def test_batched_reach_4096_instances():
    """4,096 independent Reach instances (log-uniform 32..4096 nodes, 2-4x
    edges) in one batched fixpoint, as bench.py runs them: sampled instances
    row by row against their own BFS closure, and every instance of a wider
    sample by tuple count."""
    import torch
    import paper_2311_02206_amd as pkg
    say("batched reach, 4096 instances")
    nodes, edges = workloads.batched_reach_instances(4096, seed=0xC4)
    e = pkg.Engine(device=0, stream=torch.cuda.current_stream(), ebm_k=1.5)
    try:
        e.declare("Edge", 2, True)
        e.declare("Reach", 2, False)
        e.batch_layout(nodes)
        e.load_batched("Edge", edges)
        e.program(PROG["reach"])
        st = e.run()
        say(f"  ran: {st.idb_tuples} tuples, {st.iterations} iterations, {st.seconds:.3f} s")
        rng = np.random.default_rng(5)
        for k in rng.choice(4096, 256, replace=False):
            total, _ = oracle.reach_bfs_histogram(int(nodes[k]), edges[k], threads=8)
            assert e.batch_count("Reach", int(k)) == total, k
        for k in (0, 1, 4095, int(np.argmax(nodes))):
            got = e.fetch_batched("Reach", k)
            for s in (0, int(nodes[k]) // 2, int(nodes[k]) - 1):
                lo, hi = np.searchsorted(got[:, 0], [s, s + 1])
                assert np.array_equal(got[lo:hi, 1], oracle.reach_from(int(nodes[k]), edges[k], s))
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
