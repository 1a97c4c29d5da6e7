"""Pins of the matrix-product naive evaluator (oracle/matrix_naive.py).

It is checked against brute force over all variable assignments on random
tiny programs (final sets and per-iteration deltas), against the closed
forms of Reach and of same-generation on a tree, and against the std::set
semi-naive evaluator on the CSPA-shaped program at sizes the latter
finishes in seconds.  A transposed operand, a dropped mask or a wrong
elimination order changes the brute-force results of some random program.
"""

import os

import numpy as np
import pytest

import oracle
import workloads
from oracle import matrix_naive
from test_oracle_pins import CASES, SG_RULES, as_set, brute_force, path, render

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROG = {n: open(os.path.join(ROOT, "workloads", "programs", n + ".dl")).read()
        for n in ("reach", "sg", "cspa_shaped")}
CSPA_IDB = {"ValueFlow": 2, "ValueAlias": 2, "MemoryAlias": 2}


def arrays(edb):
    return {k: np.array(sorted(v), dtype=np.uint32).reshape(-1, 2) for k, v in edb.items()}


def test_matches_brute_force_on_random_programs():
    done = 0
    for rules, edb in CASES:
        try:
            res = matrix_naive.evaluate(render(rules), arrays(edb), {"P": 2, "Q": 2},
                                        max_iterations=200)
        except NotImplementedError:
            continue
        want, wdeltas = brute_force(rules, edb)
        for n in ("P", "Q"):
            assert as_set(res.relations[n]) == want[n], render(rules)
            assert res.deltas[n] == wdeltas[n], render(rules)
        done += 1
    assert done >= 140, done


def test_sg_rules_match_brute_force():
    rng = np.random.default_rng(3)
    for _ in range(20):
        n = int(rng.integers(3, 8))
        E = {(int(a), int(b)) for a, b in rng.integers(0, n, size=(int(rng.integers(2, 12)), 2))}
        want, wdeltas = brute_force(SG_RULES, {"E": E, "F": set()})
        res = matrix_naive.evaluate(render(SG_RULES), arrays({"E": E}), {"P": 2})
        assert as_set(res.relations["P"]) == want["P"]
        assert res.deltas["P"] == wdeltas["P"]


def test_reach_closed_forms():
    for n in (2, 3, 10, 40):
        res = matrix_naive.evaluate(PROG["reach"], {"Edge": path(n)}, {"Reach": 2})
        assert len(res.relations["Reach"]) == n * (n - 1) // 2
        assert res.deltas["Reach"] == list(range(n - 1, 0, -1)) + [0]
        cyc = np.array([[i, (i + 1) % n] for i in range(n)], dtype=np.uint32)
        res = matrix_naive.evaluate(PROG["reach"], {"Edge": cyc}, {"Reach": 2})
        assert len(res.relations["Reach"]) == n * n
    res = matrix_naive.evaluate(PROG["reach"], {"Edge": np.zeros((0, 2), np.uint32)},
                                {"Reach": 2})
    assert len(res.relations["Reach"]) == 0 and res.deltas["Reach"] == [0]


def test_sg_tree_closed_form():
    E = workloads.scaled_tree(2000, seed=11)["edb"]["Edge"]
    res = matrix_naive.evaluate(PROG["sg"], {"Edge": E}, {"SG": 2})
    total, deltas = oracle.sg_tree_closed_form(E)
    assert len(res.relations["SG"]) == total
    assert res.deltas["SG"] == deltas


def test_reach_matches_bfs():
    wl = workloads.reach_er_1000()
    res = matrix_naive.evaluate(PROG["reach"], wl["edb"], {"Reach": 2})
    total, hist = oracle.reach_bfs_histogram(wl["n_nodes"], wl["edb"]["Edge"])
    assert len(res.relations["Reach"]) == total
    assert res.deltas["Reach"] == oracle.reach_deltas_from_histogram(hist)


@pytest.mark.parametrize("orient", ["literal", "by_rank", "src_zipf"])
def test_cspa_matches_semi_naive_oracle(orient):
    ids = 1 << 10
    A = workloads.zipf_pairs(ids, 390, 1.2, 0xC3, 0, orient=orient)
    D = workloads.zipf_pairs(ids, 146, 1.2, 0xC3, 1, orient=orient)
    edb = {"Assign": A, "Dereference": D}
    got = matrix_naive.evaluate(PROG["cspa_shaped"], edb, CSPA_IDB)
    want = oracle.evaluate(PROG["cspa_shaped"], edb, CSPA_IDB)
    for n in CSPA_IDB:
        assert np.array_equal(got.relations[n], want.relations[n]), n
        assert got.deltas[n] == want.deltas[n], n
    assert got.iterations == want.iterations


def test_unsupported_forms_raise():
    with pytest.raises(NotImplementedError):
        # z and w each meet three other variables: no pairwise elimination
        matrix_naive.evaluate("P(x, y) :- E(z, x), E(z, y), E(z, w), E(w, x), E(w, y).",
                              {"E": path(4)}, {"P": 2})
    with pytest.raises(NotImplementedError):
        matrix_naive.evaluate("P(x, y, z) :- E(x, y), E(y, z).", {"E": path(4)}, {"P": 3})


def _mismatches():
    bad = 0
    for rules, edb in CASES[:80]:
        want, wdeltas = brute_force(rules, edb)
        res = matrix_naive.evaluate(render(rules), arrays(edb), {"P": 2, "Q": 2},
                                    max_iterations=200)
        bad += any(as_set(res.relations[n]) != want[n] or res.deltas[n] != wdeltas[n]
                   for n in ("P", "Q"))
    return bad


@pytest.mark.parametrize("plant", ["no_transpose", "drop_mask", "jacobi_to_gauss"])
def test_planted_mistakes_are_caught(monkeypatch, plant):
    """Plant a plausible mistake in the evaluator; the brute-force pins must
    notice it."""
    if plant == "no_transpose":
        monkeypatch.setattr(matrix_naive._Factor, "oriented", lambda self, first: self.arr)
    elif plant == "drop_mask":
        real = matrix_naive._eliminate

        def no_mask(factors, z):
            # forget the one-variable conjuncts on z when z is also in a matrix
            if any(len(f.vars) == 2 and z in f.vars for f in factors):
                factors = [f for f in factors if not (len(f.vars) == 1 and z in f.vars)]
            return real(factors, z)
        monkeypatch.setattr(matrix_naive, "_eliminate", no_mask)
    else:
        real_rule = matrix_naive._eval_rule

        def gauss(rule, mats, k):
            out = real_rule(rule, mats, k)
            name = rule.head[0]
            if name in mats and name in ("P", "Q"):
                mats[name] = mats[name] | out   # later rules see this rule's output
            return out
        monkeypatch.setattr(matrix_naive, "_eval_rule", gauss)
    assert _mismatches() > 0


def test_cspa_2p15_fixture_is_consistent():
    """The stored 2^15-id CSPA reference (written by
    tests/golden/make_cspa_2p15.py from the matrix evaluator) is internally
    consistent: every relation's size is the sum of its per-iteration
    deltas, and the last iteration is the empty one."""
    import json
    fx = json.load(open(os.path.join(ROOT, "tests", "golden", "cspa_2p15.json")))
    assert set(fx["relations"]) == set(CSPA_IDB)
    for n, r in fx["relations"].items():
        assert len(r["deltas"]) == fx["iterations"]
        assert sum(r["deltas"]) == r["size"] and r["deltas"][-1] == 0
        assert len(r["sha256"]) == 64
