"""Pins for the oracle: checks against things other than the oracle itself.

* the paper's worked examples (tests/golden/, each citing its passage);
* brute force: the immediate-consequence operator applied by enumerating
  every variable assignment over the active domain (tiny inputs), iterated
  to its least fixpoint, on random programs;
* breadth-first search (scipy.sparse.csgraph) for Reach, including the
  per-iteration delta sizes implied by shortest distances;
* closed forms: Reach on paths, cycles, complete digraphs; SG on trees;
* invariants: closure idempotence, transitivity, SG symmetry and
  irreflexivity, sum of deltas equals the final size, row-order invariance;
* planted mistakes: each one must make at least one pin fail.
"""

import itertools
import os
import random

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REACH = open(os.path.join(ROOT, "workloads", "programs", "reach.dl")).read()
SG = open(os.path.join(ROOT, "workloads", "programs", "sg.dl")).read()


def as_set(rows):
    return {tuple(int(x) for x in r) for r in rows}


def read_fixture(name):
    out = {}
    for line in open(os.path.join(ROOT, "tests", "golden", name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, val = line.split(":", 1)
        out.setdefault(key.strip(), []).append(val.strip())
    return out


def parse_tuples(s):
    return [tuple(int(x) for x in t.split()) for t in s.split(",")]


# ------------------------------------------------------------ paper examples

def test_sg_paper_example():
    fx = read_fixture("sg_paper_example.txt")
    edges = np.array(parse_tuples(fx["edges"][0]), dtype=np.uint32)
    res = oracle.evaluate(SG, {"Edge": edges}, {"SG": 2}, history=True)
    dh, nh = res.delta_history["SG"], res.new_history["SG"]
    # keys carry the iteration in the key text: "delta_member 0"
    for key, vals in fx.items():
        kind, _, it = key.partition(" ")
        if kind not in ("delta_member", "new_member", "full_before"):
            continue
        it = int(it)
        for v in vals:
            t = tuple(int(x) for x in v.split())
            if kind == "delta_member":
                assert t in as_set(dh[it]), (kind, it, t)
            elif kind == "new_member":
                assert t in as_set(nh[it]), (kind, it, t)
            else:
                full_before = set().union(*[as_set(d) for d in dh[:it]])
                assert t in full_before, (kind, it, t)
    assert res.iterations == int(fx["iterations"][0])
    assert res.deltas["SG"][-1] == 0
    # paper: the new set of the last iteration is non-empty and all duplicates
    assert len(nh[-1]) > 0
    # and the whole run agrees with brute force on the same graph
    want, wdeltas = brute_force(SG_RULES, {"E": as_set(edges)})
    assert as_set(res.relations["SG"]) == want["P"]
    assert res.deltas["SG"] == wdeltas["P"]


def test_foobar_paper_example():
    fx = read_fixture("foobar_paper_example.txt")
    foo = np.array(parse_tuples(fx["foo"][0]), dtype=np.uint32)
    bar = np.array(parse_tuples(fx["bar"][0]), dtype=np.uint32)
    prog = "Foobar(c, d) :- Foo(a, b, c), Bar(a, b, d)."
    res = oracle.evaluate(prog, {"Foo": foo, "Bar": bar}, {"Foobar": 2})
    got = as_set(res.relations["Foobar"])
    for v in fx["expect_member"]:
        assert tuple(int(x) for x in v.split()) in got
    assert got == {(5, 1), (2, 1)}


def test_sorted_index_reading():
    """The reading of the sorted-index example: join column first, then the
    remaining columns in order; the stated lexicographic order wins."""
    fx = read_fixture("sorted_index_example.txt")
    tup = np.array(parse_tuples(fx["tuples"][0]))
    jc = int(fx["join_column"][0])
    rest = [c for c in range(tup.shape[1]) if c != jc]
    reordered = [tuple([t[jc]] + [t[c] for c in rest]) for t in tup.tolist()]
    order = sorted(range(len(reordered)), key=lambda i: reordered[i])
    assert order == [int(x) for x in fx["expect_order"][0].split()]


# ----------------------------------------------------------------- brute force

VARS = "abcd"


def random_program(rng):
    """Random positive program over EDB E, F and IDB P, Q (all binary)."""
    rels = ["E", "F", "P", "Q"]
    rules = []
    for _ in range(rng.randint(2, 4)):
        nb = rng.randint(1, 3)
        body = []
        for _ in range(nb):
            body.append((rng.choice(rels), rng.choice(VARS), rng.choice(VARS)))
        bvars = sorted({v for a in body for v in a[1:]})
        head = (rng.choice(["P", "Q"]), rng.choice(bvars), rng.choice(bvars))
        filt = None
        if len(bvars) >= 2 and rng.random() < 0.4:
            x, y = rng.sample(bvars, 2)
            filt = (x, y)
        rules.append((head, body, filt))
    # make sure something seeds the IDBs
    rules.append((("P", "a", "b"), [("E", "a", "b")], None))
    return rules


def render(rules):
    lines = []
    for head, body, filt in rules:
        parts = [f"{r}({x}, {y})" for r, x, y in body]
        if filt:
            parts.append(f"{filt[0]} != {filt[1]}")
        lines.append(f"{head[0]}({head[1]}, {head[2]}) :- " + ", ".join(parts) + ".")
    return "\n".join(lines)


def brute_force(rules, edb):
    """Least fixpoint by iterating T_P over all assignments of the active
    domain.  Returns (final sets, per-iteration delta sizes)."""
    edb = dict(edb)
    edb.setdefault("F", set())
    dom = sorted({x for rows in edb.values() for t in rows for x in t})
    full = {"P": set(), "Q": set()}
    rel = lambda n: edb[n] if n in edb else full[n]
    deltas = {"P": [], "Q": []}
    while True:
        fresh = {"P": set(), "Q": set()}
        for head, body, filt in rules:
            vs = sorted({v for a in body for v in a[1:]})
            for vals in itertools.product(dom, repeat=len(vs)):
                b = dict(zip(vs, vals))
                if all((b[x], b[y]) in rel(r) for r, x, y in body):
                    if filt and b[filt[0]] == b[filt[1]]:
                        continue
                    fresh[head[0]].add((b[head[1]], b[head[2]]))
        total = 0
        for n in ("P", "Q"):
            d = fresh[n] - full[n]
            deltas[n].append(len(d))
            total += len(d)
        for n in ("P", "Q"):
            full[n] |= fresh[n]
        if total == 0:
            return full, deltas


# the SG program (Section 2) in the brute-force rule format (SG = P, Edge = E)
SG_RULES = [(("P", "x", "y"), [("E", "p", "x"), ("E", "p", "y")], ("x", "y")),
            (("P", "x", "y"), [("E", "a", "x"), ("P", "a", "b"), ("E", "b", "y")], ("x", "y"))]


def random_edb(rng):
    n = rng.randint(2, 5)
    out = {}
    for name in ("E", "F"):
        m = rng.randint(0, 7)
        out[name] = {(rng.randrange(n), rng.randrange(n)) for _ in range(m)}
    return out


def run_oracle_on(rules, edb, mode="semi_naive", plant=0):
    arr = {k: np.array(sorted(v), dtype=np.uint32).reshape(-1, 2) for k, v in edb.items()}
    return oracle.evaluate(render(rules), arr, {"P": 2, "Q": 2}, mode=mode, plant=plant,
                           max_iterations=200)


def brute_force_cases(n=150, seed=1234):
    rng = random.Random(seed)
    return [(random_program(rng), random_edb(rng)) for _ in range(n)]


CASES = brute_force_cases()


def test_semi_naive_matches_brute_force():
    for rules, edb in CASES:
        want, wdeltas = brute_force(rules, edb)
        res = run_oracle_on(rules, edb)
        for n in ("P", "Q"):
            assert as_set(res.relations[n]) == want[n], render(rules)
            assert res.deltas[n] == wdeltas[n], render(rules)


def test_naive_mode_matches_brute_force():
    for rules, edb in CASES[:60]:
        want, wdeltas = brute_force(rules, edb)
        res = run_oracle_on(rules, edb, mode="naive")
        for n in ("P", "Q"):
            assert as_set(res.relations[n]) == want[n]
            assert res.deltas[n] == wdeltas[n]


# ------------------------------------------------------------------ Reach pins

def scipy_reach(n, edges):
    """Reach and per-distance counts from scipy's unweighted shortest paths."""
    if len(edges) == 0:
        return set(), []
    A = csr_matrix((np.ones(len(edges)), (edges[:, 0], edges[:, 1])), shape=(n, n))
    D = shortest_path(A, unweighted=True, directed=True)
    pairs = {}
    for s in range(n):
        for t in range(n):
            if s != t and np.isfinite(D[s, t]):
                pairs[(s, t)] = int(D[s, t])
    # (s, s): shortest cycle through s = min over in-edges (u, s) of D[s, u] + 1
    for u, s in edges.tolist():
        if np.isfinite(D[s, u]):
            d = int(D[s, u]) + 1
            if (s, s) not in pairs or pairs[(s, s)] > d:
                pairs[(s, s)] = d
    maxd = max(pairs.values())
    hist = [0] * (maxd + 1)
    for d in pairs.values():
        hist[d] += 1
    return set(pairs), hist[1:] + [0]


@pytest.mark.parametrize("seed", range(6))
def test_reach_matches_scipy_bfs(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 60))
    m = int(rng.integers(0, 3 * n))
    edges = np.unique(rng.integers(0, n, size=(m, 2)).astype(np.uint32), axis=0)
    res = oracle.evaluate(REACH, {"Edge": edges.reshape(-1, 2)}, {"Reach": 2})
    want, wdeltas = scipy_reach(n, edges.reshape(-1, 2))
    assert as_set(res.relations["Reach"]) == want
    if want:
        assert res.deltas["Reach"] == wdeltas


def test_reach_er1000_matches_bfs_histogram():
    wl = workloads.reach_er_1000()
    res = oracle.evaluate(REACH, wl["edb"], {"Reach": 2})
    total, hist = oracle.reach_bfs_histogram(wl["n_nodes"], wl["edb"]["Edge"])
    assert len(res.relations["Reach"]) == total
    assert res.deltas["Reach"] == oracle.reach_deltas_from_histogram(hist)
    # sampled sources, compared row by row
    R = res.relations["Reach"]
    for s in (0, 17, 500, 999):
        want = oracle.reach_from(wl["n_nodes"], wl["edb"]["Edge"], s)
        got = R[R[:, 0] == s][:, 1]
        assert np.array_equal(got, want)


def test_bfs_checker_matches_scipy():
    rng = np.random.default_rng(7)
    for _ in range(5):
        n = int(rng.integers(5, 80))
        edges = np.unique(rng.integers(0, n, size=(2 * n, 2)).astype(np.uint32), axis=0)
        total, hist = oracle.reach_bfs_histogram(n, edges, threads=3)
        want, wdeltas = scipy_reach(n, edges)
        assert total == len(want)
        assert oracle.reach_deltas_from_histogram(hist) == wdeltas


def path(n):
    return np.array([[i, i + 1] for i in range(n - 1)], dtype=np.uint32).reshape(-1, 2)


def test_reach_closed_forms():
    for n in (2, 3, 10, 40):
        res = oracle.evaluate(REACH, {"Edge": path(n)}, {"Reach": 2})
        assert len(res.relations["Reach"]) == n * (n - 1) // 2
        # n-1 productive iterations (distances 1..n-1) plus the empty one
        assert res.deltas["Reach"] == list(range(n - 1, 0, -1)) + [0]
        cyc = np.array([[i, (i + 1) % n] for i in range(n)], dtype=np.uint32)
        res = oracle.evaluate(REACH, {"Edge": cyc}, {"Reach": 2})
        assert len(res.relations["Reach"]) == n * n
        comp = np.array([[i, j] for i in range(n) for j in range(n) if i != j], dtype=np.uint32)
        res = oracle.evaluate(REACH, {"Edge": comp}, {"Reach": 2})
        assert len(res.relations["Reach"]) == n * n
    res = oracle.evaluate(REACH, {"Edge": np.zeros((0, 2), dtype=np.uint32)}, {"Reach": 2})
    assert len(res.relations["Reach"]) == 0 and res.deltas["Reach"] == [0]
    res = oracle.evaluate(REACH, {"Edge": np.array([[7, 7]], dtype=np.uint32)}, {"Reach": 2})
    assert as_set(res.relations["Reach"]) == {(7, 7)}


def test_reach_invariants():
    wl = workloads.scaled_rmat(8, 600, seed=3)
    E = wl["edb"]["Edge"]
    res = oracle.evaluate(REACH, {"Edge": E}, {"Reach": 2})
    R = res.relations["Reach"]
    assert sum(res.deltas["Reach"]) == len(R)
    # sorted and unique
    key = (R[:, 0].astype(np.uint64) << np.uint64(32)) | R[:, 1]
    assert np.all(np.diff(key.astype(np.int64)) > 0)
    # idempotence: the closure of the closure is itself
    res2 = oracle.evaluate(REACH, {"Edge": R}, {"Reach": 2})
    assert np.array_equal(res2.relations["Reach"], R)
    # transitivity on sampled triples
    S = as_set(R)
    rng = np.random.default_rng(0)
    for i in rng.integers(0, len(R), 200):
        a, b = R[i]
        for c in R[R[:, 0] == b][:, 1][:5]:
            assert (int(a), int(c)) in S
    # row order of the EDB does not matter
    perm = rng.permutation(len(E))
    res3 = oracle.evaluate(REACH, {"Edge": np.concatenate([E[perm], E[:10]])}, {"Reach": 2})
    assert np.array_equal(res3.relations["Reach"], R)
    assert res3.deltas["Reach"] == res.deltas["Reach"]


# --------------------------------------------------------------------- SG pins

@pytest.mark.parametrize("n", [1, 2, 7, 60, 400])
def test_sg_tree_closed_form(n):
    E = workloads.random_tree(n, seed=n)
    res = oracle.evaluate(SG, {"Edge": E}, {"SG": 2})
    total, deltas = oracle.sg_tree_closed_form(E) if len(E) else (0, [0])
    assert len(res.relations["SG"]) == total
    assert res.deltas["SG"] == deltas
    S = res.relations["SG"]
    assert np.all(S[:, 0] != S[:, 1])
    assert as_set(S) == {(b, a) for a, b in as_set(S)}


def test_sg_tree_closed_form_matches_depth_definition():
    """The closed form itself against its definition (same depth >= 1)."""
    E = workloads.random_tree(300, seed=9)
    depth = {0: 0}
    for p, c in E.tolist():
        depth[c] = depth[p] + 1   # breadth-first ids: parents come first
    want = {(x, y) for x in depth for y in depth if x != y and depth[x] == depth[y] >= 1}
    total, _ = oracle.sg_tree_closed_form(E)
    assert total == len(want)
    res = oracle.evaluate(SG, {"Edge": E}, {"SG": 2})
    assert as_set(res.relations["SG"]) == want


# --------------------------------------------------------------- planted bugs

# A program where a rule with two IDB atoms needs its second delta variant:
# Q(1,4) joins the old P(1,2) with the later P(2,4).
TWO_VARIANT_RULES = [(("P", "a", "b"), [("E", "a", "b")], None),
                     (("P", "a", "b"), [("P", "a", "c"), ("F", "c", "b")], None),
                     (("Q", "a", "b"), [("P", "a", "c"), ("P", "c", "b")], None)]
TWO_VARIANT_EDB = {"E": {(1, 2), (2, 3)}, "F": {(3, 4), (4, 5), (5, 6)}}


def test_two_variant_case():
    want, wdeltas = brute_force(TWO_VARIANT_RULES, TWO_VARIANT_EDB)
    assert (1, 4) in want["Q"]
    res = run_oracle_on(TWO_VARIANT_RULES, TWO_VARIANT_EDB)
    for n in ("P", "Q"):
        assert as_set(res.relations[n]) == want[n]
        assert res.deltas[n] == wdeltas[n]


def pins_pass(plant):
    """Runs a subset of the pins against an oracle with a planted mistake."""
    try:
        for rules, edb in [(TWO_VARIANT_RULES, TWO_VARIANT_EDB)] + CASES[:80]:
            want, wdeltas = brute_force(rules, edb)
            res = run_oracle_on(rules, edb, plant=plant)
            for n in ("P", "Q"):
                if as_set(res.relations[n]) != want[n] or res.deltas[n] != wdeltas[n]:
                    return False
        fx = read_fixture("sg_paper_example.txt")
        edges = np.array(parse_tuples(fx["edges"][0]), dtype=np.uint32)
        res = oracle.evaluate(SG, {"Edge": edges}, {"SG": 2}, plant=plant, max_iterations=50)
        want, wdeltas = brute_force(SG_RULES, {"E": as_set(edges)})
        if as_set(res.relations["SG"]) != want["P"] or res.deltas["SG"] != wdeltas["P"]:
            return False
        E = path(12)
        res = oracle.evaluate(REACH, {"Edge": E}, {"Reach": 2}, plant=plant, max_iterations=50)
        if res.deltas["Reach"] != list(range(11, 0, -1)) + [0]:
            return False
    except RuntimeError:
        return False
    return True


def test_pins_pass_unplanted():
    assert pins_pass(0)


@pytest.mark.parametrize("plant", [1, 3, 4, 5, 6])
def test_planted_mistake_is_caught(plant):
    assert not pins_pass(plant)


NONLINEAR = "T(x, y) :- E(x, y).\nT(x, y) :- T(x, z), T(z, y)."


@pytest.mark.parametrize("seed", range(6))
def test_doubling_deltas_match_semi_naive(seed):
    """The nonlinear closure's per-iteration deltas implied by the distance
    histogram (after iteration i exactly the pairs at distance <= 2^i)
    equal the std::set evaluator's, and so does the final relation."""
    E = workloads.erdos_renyi(300, 330 + 40 * seed, seed)
    res = oracle.evaluate(NONLINEAR, {"E": E}, {"T": 2})
    total, hist = oracle.reach_bfs_histogram(300, E)
    assert len(res.relations["T"]) == total
    assert res.deltas["T"] == oracle.doubling_deltas_from_histogram(hist)


def test_doubling_deltas_on_a_path():
    """A directed path of n nodes: distance d has n - d pairs, so iteration
    i adds the distances 2^(i-1)+1 .. 2^i."""
    for n in (2, 3, 5, 9, 33):
        res = oracle.evaluate(NONLINEAR, {"E": path(n)}, {"T": 2})
        want = [n - 1]
        lo = 2
        while lo <= n - 1:
            hi = min(2 * (lo - 1), n - 1)
            want.append(sum(n - d for d in range(lo, hi + 1)))
            lo = hi + 1
        assert res.deltas["T"] == want + [0]
        _, hist = oracle.reach_bfs_histogram(n, path(n))
        assert oracle.doubling_deltas_from_histogram(hist) == want + [0]
